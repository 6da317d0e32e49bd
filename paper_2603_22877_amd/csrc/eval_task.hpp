// One wavefront task of the diagram passes, shared by the per-call kernel and the fused
// solver. A task is 64 lanes, each a (constraint position, restart) pair of one bucket, so
// the diagram shape is uniform across the wave: node records come through the scalar unit
// and each lane keeps its messages in its own LDS column ([row][lane] layout).
//
// State access and gradient accumulation are template policies: global strided views with
// L2 atomics (per-call path) or LDS-resident state with LDS atomics (fused solver).
#pragma once
#include <type_traits>

#include "kernels_common.hpp"

namespace fsmt {

// Device pointers of one compiled instance.
struct TabView {
    cptr<TplInfo> tpl;
    cptr<Node> nodes;
    cptr<BucketInfo> bucket;
    cptr<int32_t> bucket_start;
    cptr<int32_t> task_bucket;
    cptr<AtomRec> arec;
    cptr<int32_t> pos_con;
    cptr<int32_t> sup;
    cptr<int32_t> con_bucket;
    cptr<int32_t> con_local;
    cptr<GdInfo> gd;
    cptr<GdForm> gdf;
    cptr<SlimRec> srec;
    cptr<int32_t> atom_ptr;
    cptr<int32_t> atom_var;
    cptr<double> atom_coef;
    cptr<double> atom_rhs;
    cptr<double> atom_scale;
    cptr<uint8_t> atom_strict;
    cptr<float> real_lo;
    cptr<float> real_hi;
    int32_t n_bool, n_real, n_cons, n_pos, n_buckets, pad;

    static TabView of(const fsmt_xbdd *h) {
        TabView t;
        t.tpl = as_cptr(h->d.tpl);
        t.nodes = as_cptr(h->d.nodes);
        t.bucket = as_cptr(h->d.bucket);
        t.bucket_start = as_cptr(h->d.bucket_start);
        t.task_bucket = as_cptr(h->d.task_bucket);
        t.arec = as_cptr(h->d.arec);
        t.pos_con = as_cptr(h->d.pos_con);
        t.sup = as_cptr(h->d.sup);
        t.con_bucket = as_cptr(h->d.con_bucket);
        t.con_local = as_cptr(h->d.con_local);
        t.gd = as_cptr(h->d.gd);
        t.gdf = as_cptr(h->d.gdf);
        t.srec = as_cptr(h->d.srec);
        t.atom_ptr = as_cptr(h->d.atom_ptr);
        t.atom_var = as_cptr(h->d.atom_var);
        t.atom_coef = as_cptr(h->d.atom_coef);
        t.atom_rhs = as_cptr(h->d.atom_rhs);
        t.atom_scale = as_cptr(h->d.atom_scale);
        t.atom_strict = as_cptr(h->d.atom_strict);
        t.real_lo = as_cptr(h->d.real_lo);
        t.real_hi = as_cptr(h->d.real_hi);
        t.n_bool = h->n_bool;
        t.n_real = h->n_real;
        t.n_cons = h->n_cons;
        t.n_pos = h->n_pos;
        t.n_buckets = h->n_buckets;
        t.pad = 0;
        return t;
    }
};

// ---- state policies
struct GlobalState {
    View a, b;
    __device__ __forceinline__ float av(int r, int i) const { return a.at(r, i); }
    __device__ __forceinline__ float bv(int r, int j) const { return b.at(r, j); }
};
struct LdsState {
    const float *a, *b;
    __device__ __forceinline__ float av(int, int i) const { return a[i]; }
    __device__ __forceinline__ float bv(int, int j) const { return b[j]; }
};

// ---- gradient accumulation policies
// Every lane calls add_a / add_b at the same points (uniform control flow); a lane with
// nothing to add passes var < 0.
//
// Global memory: device-scope float atomics are performed past the per-XCD L2, so equal
// (variable, restart) targets held by different constraint groups of the wave (lanes
// rpad apart) are first merged by a shuffle butterfly; one atomic per remaining target.
struct GlobalScatter {
    View ga, gb;
    int rpad;   // lanes per constraint group (64: one group, nothing to merge)
    __device__ __forceinline__ void merge(int &var, float &val, int lane) const {
        for (int off = rpad; off < 64; off <<= 1) {
            const int pv = __shfl_xor(var, off, 64);
            const float pval = __shfl_xor(val, off, 64);
            if (pv == var && var >= 0) {
                if ((lane & off) == 0) val += pval; else val = 0.0f;
            }
        }
    }
    __device__ __forceinline__ void add_a(int r, int i, float g, int lane) const {
        merge(i, g, lane);
        if (i >= 0 && g != 0.0f) atomic_add_f32(&ga.at(r, i), g);
    }
    __device__ __forceinline__ void add_b(int r, int j, float g, int lane) const {
        merge(j, g, lane);
        if (j >= 0 && g != 0.0f) atomic_add_f32(&gb.at(r, j), g);
    }
    // for divergent call sites (no merging)
    __device__ __forceinline__ void add_b_direct(int r, int j, float g) const { atomic_add_f32(&gb.at(r, j), g); }
    __device__ __forceinline__ void add_a_direct(int r, int i, float g) const { atomic_add_f32(&ga.at(r, i), g); }
};
// LDS: the fused solver's gradient lives in LDS and its atomics stay on the CU.
struct LdsScatter {
    float *ga, *gb;
    __device__ __forceinline__ void add_a(int, int i, float g, int) const {
        if (i >= 0 && g != 0.0f) atomicAdd(ga + i, g);
    }
    __device__ __forceinline__ void add_b(int, int j, float g, int) const {
        if (j >= 0 && g != 0.0f) atomicAdd(gb + j, g);
    }
    __device__ __forceinline__ void add_b_direct(int, int j, float g) const { atomicAdd(gb + j, g); }
};

// z = q.b - q0 of atom k for restart r (exact order, see atom_z_exact).
template <class St>
__device__ __forceinline__ double atom_z_state(const TabView &T, int k, const St &st, int r) {
#pragma clang fp contract(off)
    double acc = 0.0;
    const int e1 = T.atom_ptr[k + 1];
    for (int e = T.atom_ptr[k]; e < e1; ++e) {
        const double prod = T.atom_coef[e] * (double)st.bv(r, T.atom_var[e]);
        acc = acc + prod;
    }
    return acc - T.atom_rhs[k];
}

// z of an inline atom record: the same multiply-then-add sequence as the CSR form.
template <class St>
__device__ __forceinline__ double rec_z(const AtomRec &a, const St &st, int r) {
#pragma clang fp contract(off)
    double acc = 0.0;
    const double p0 = (double)a.c0 * (double)st.bv(r, a.v0);
    acc = acc + p0;
    if (a.flags & 2u) {
        const double p1 = (double)a.c1 * (double)st.bv(r, a.v1);
        acc = acc + p1;
    }
    return acc - (double)a.rhs;
}

__device__ __forceinline__ AtomRec load_rec(cptr<AtomRec> p) {
    const i32x4 x = ((cptr<i32x4>)p)[0];
    const i32x4 z = ((cptr<i32x4>)p)[1];
    AtomRec a;
    a.v0 = x.x;
    a.v1 = x.y;
    a.c0 = __int_as_float(x.z);
    a.c1 = __int_as_float(x.w);
    a.rhs = __int_as_float(z.x);
    a.scale = __int_as_float(z.y);
    a.atom = z.z;
    a.flags = (uint32_t)z.w;
    return a;
}

// Find the bucket containing position pos (uniform across the wave).
__device__ __forceinline__ int find_bucket(cptr<int32_t> start, int nb, int pos) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (__builtin_amdgcn_readfirstlane(start[mid]) <= pos) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Per-wave LDS scratch: M[NN][64], Bm[NN][64], P[SS][64], Q[SS][64], D[SS][64], G[SS][64].
struct WaveScratch {
    float *M, *Bm, *P, *Q, *D, *G;
    __device__ __forceinline__ static WaveScratch at(float *base, int NN, int SS) {
        WaveScratch s;
        s.M = base;
        s.Bm = s.M + NN * 64;
        s.P = s.Bm + NN * 64;
        s.Q = s.P + SS * 64;
        s.D = s.Q + SS * 64;
        s.G = s.D + SS * 64;
        return s;
    }
    __host__ __device__ static size_t bytes(int NN, int SS) { return (size_t)(2 * NN + 4 * SS) * 64 * sizeof(float); }
};

struct TaskCtx {
    BucketInfo B;         // bucket record with the template fields
    cptr<int32_t> sup;    // this lane's support column
    cptr<AtomRec> rec;    // this lane's first inline atom record (or null)
    int local;            // position inside the bucket
    int c;                // original constraint id (or -1)
    int r;
    bool valid;
};

// Locate the task: pos is this lane's position, all lanes of the wave in one bucket.
__device__ __forceinline__ TaskCtx task_ctx(const TabView &T, int pos, int r, bool r_ok) {
    TaskCtx t;
    const int pos0 = __builtin_amdgcn_readfirstlane(pos);
    const int bk = __builtin_amdgcn_readfirstlane(T.task_bucket[pos0 >> 6]);
    t.B = load_bucket(T.bucket + bk);
    const int local = pos - t.B.pos_begin;
    t.sup = T.sup + t.B.sup_base + local;
    t.rec = t.B.arec_base >= 0 ? T.arec + t.B.arec_base + local : nullptr;
    t.local = local;
    t.c = T.pos_con[pos];
    t.r = r;
    t.valid = (t.c >= 0) && r_ok;
    return t;
}

// ---- message stores
// A store holds one lane's forward masses M and reverse probabilities Bm per node (plus the
// two terminals) and P = P[literal True], Q = 1 - P, D = dp/dz, G = dP[False]/dp per slot.
//
// RegMsgs keeps them in VGPRs: the diagram size is bounded at compile time, so every loop
// over nodes or slots unrolls (guarded by the bucket's actual sizes), static indices become
// plain registers, and the wave-uniform child and slot indices read from a node record
// address the arrays through gfx950's GPR indexing. The node chain then runs at register
// latency and no LDS is needed. LdsMsgs keeps them in the wave's LDS columns ([row][lane])
// for diagrams of any size.
template <int NM, int SM>
struct RegMsgs {
    static constexpr int kNodes = NM, kSlots = SM;
    // Node arrays hold the NM nodes, the two terminals and a spare entry that absorbs the
    // updates of iterations past the diagram's size (index kTrashNode); slot arrays hold a
    // spare slot (kTrashSlot) likewise. At least 9 elements per array: the compiler lowers
    // a uniform dynamic index into a shorter register array as a compare/select per
    // element, into a longer one as a single indexed move (GPR indexing).
    static constexpr int kTrashNode = NM + 2, kTrashSlot = SM;
    static constexpr int kArrNodes = NM + 3 < 9 ? 9 : NM + 3, kArrSlots = SM + 1 < 9 ? 9 : SM + 1;
    static constexpr bool kInlineOnly = true;   // every atom slot has an inline record
    // the arrays are separate locals of the kernel (see bind_msgs): a single aggregate
    // indexed dynamically would not be split into registers
    float *m_, *b_, *p_, *q_, *d_, *g_;
    __device__ __forceinline__ float &M(int v) { return m_[v]; }
    __device__ __forceinline__ float &Bm(int v) { return b_[v]; }
    __device__ __forceinline__ float &P(int s) { return p_[s]; }
    __device__ __forceinline__ float &Q(int s) { return q_[s]; }
    __device__ __forceinline__ float &D(int s) { return d_[s]; }
    __device__ __forceinline__ float &G(int s) { return g_[s]; }
};

struct LdsMsgs {
    static constexpr int kNodes = 0, kSlots = 0;   // unbounded
    static constexpr int kArrNodes = 1, kArrSlots = 1;
    static constexpr int kTrashNode = 0, kTrashSlot = 0;
    static constexpr bool kInlineOnly = false;      // inline records or the CSR atom table
    WaveScratch W;
    int lane;
    __device__ __forceinline__ float &M(int v) { return W.M[v * 64 + lane]; }
    __device__ __forceinline__ float &Bm(int v) { return W.Bm[v * 64 + lane]; }
    __device__ __forceinline__ float &P(int s) { return W.P[s * 64 + lane]; }
    __device__ __forceinline__ float &Q(int s) { return W.Q[s * 64 + lane]; }
    __device__ __forceinline__ float &D(int s) { return W.D[s * 64 + lane]; }
    __device__ __forceinline__ float &G(int s) { return W.G[s * 64 + lane]; }
};

// for (i = lo; i < n; ++i) f(i), fully unrolled over [lo, K) when the bound K is static
template <int K, class F>
__device__ __forceinline__ void for_up(int lo, int n, F &&f) {
    if constexpr (K > 0) {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i >= lo && i < n) f(i);
    } else {
        for (int i = lo; i < n; ++i) f(i);
    }
}
// for (i = n - 1; i >= 0; --i) f(i)
template <int K, class F>
__device__ __forceinline__ void for_down(int n, F &&f) {
    if constexpr (K > 0) {
#pragma unroll
        for (int i = K - 1; i >= 0; --i)
            if (i < n) f(i);
    } else {
        for (int i = n - 1; i >= 0; --i) f(i);
    }
}

// Literal probability of one atom slot under Gaussian smoothing (Eq. "sampling"):
// p = erfc(u) / 2 with u = kappa * scale * z, z = q.b - q0 and scale = 1 / (sqrt 2 |q|)
// fixed at compile time, and its derivative dp/dz. Hard mode (kappa = inf) is the
// indicator of the atom at b.
// erfc(x) for x >= 0, and exp(-x^2), by the Chebyshev fit of Numerical Recipes (Press,
// Teukolsky, Vetterling, Flannery, 2nd ed., Sec. 6.2, "erfcc"):
//   t = 1 / (1 + x/2),  erfc(x) = t exp(-x^2 + P(t)),  P a degree-9 polynomial,
// fractional error below 1.2e-7 for all x >= 0. Float32 evaluation with the hardware
// reciprocal and base-2 exponential adds a few ulps where erfc is not negligible (the
// exponent's rounding grows with x^2, i.e. where erfc(x) < 1e-8); about 20 instructions for
// both values against ~55 for the library erfcf plus expf.
__device__ __forceinline__ float erfc_nr(float x, float &emx2) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
    float pt = 0.17087277f;
    pt = fmaf(pt, t, -0.82215223f);
    pt = fmaf(pt, t, 1.48851587f);
    pt = fmaf(pt, t, -1.13520398f);
    pt = fmaf(pt, t, 0.27886807f);
    pt = fmaf(pt, t, -0.18628806f);
    pt = fmaf(pt, t, 0.09678418f);
    pt = fmaf(pt, t, 0.37409196f);
    pt = fmaf(pt, t, 1.00002368f);
    pt = fmaf(pt, t, -1.26551223f);
    const float x2 = x * x;
    constexpr float kLog2e = 1.44269504088896340736f;
    emx2 = __builtin_amdgcn_exp2f(-x2 * kLog2e);
    return t * __builtin_amdgcn_exp2f((pt - x2) * kLog2e);
}

__device__ __forceinline__ void atom_literal(double z, double scale, bool strict, double kappa, bool hard,
                                             float &p, float &q, float &d) {
    if (hard) {
        const bool tr = strict ? (z < 0.0) : (z <= 0.0);
        p = tr ? 1.0f : 0.0f;
        q = tr ? 0.0f : 1.0f;
        d = 0.0f;
    } else {
        const double ks = kappa * scale;
        const float u = (float)(z * ks);
        float emu2;
        const float e = 0.5f * erfc_nr(fabsf(u), emu2);   // the smaller of p, 1-p
        p = (u >= 0.0f) ? e : 1.0f - e;
        q = (u >= 0.0f) ? 1.0f - e : e;
        if (u != u) { p = u; q = u; }                    // NaN in, NaN out
        d = -(float)(ks * 0.56418958354775628695) * emu2;   // dp/dz = -k s/sqrt(pi) e^-u^2
    }
}

// Literal probabilities and the forward pass; returns P[c False] (0 for invalid lanes).
template <class St, class Ms>
__device__ __forceinline__ float task_forward(const TabView &T, const TaskCtx &t, const St &st, double kappa,
                                              bool hard, Ms &W) {
    constexpr int KN = Ms::kNodes, KS = Ms::kSlots;
    const int N = t.B.n_nodes, S = t.B.n_slots, NB = t.B.n_bslots;
    const int64_t np = t.B.n_pos;
    // the first Boolean id and the first atom record are requested together before any
    // slot is evaluated, so their latencies overlap (a clause has one of each)
    const int id0 = NB > 0 ? t.sup[0] : 0;
    AtomRec rec0;
    const bool has_rec0 = (Ms::kInlineOnly || t.rec) && S > NB;
    if (has_rec0) rec0 = load_rec(t.rec);
    for_up<KS>(0, NB, [&](int s) {
        const float av = t.valid ? st.av(t.r, s == 0 ? id0 : t.sup[(int64_t)s * np]) : 0.0f;
        W.P(s) = (1.0f - av) * 0.5f;
        W.Q(s) = (1.0f + av) * 0.5f;
    });
    for_up<KS>(NB, S, [&](int s) {
        float p = 0.5f, q = 0.5f, d = 0.0f;
        if (t.valid) {
            if (Ms::kInlineOnly || t.rec) {
                const AtomRec a = s == NB ? rec0 : load_rec(t.rec + (int64_t)(s - NB) * np);
                atom_literal(rec_z(a, st, t.r), (double)a.scale, (a.flags & 1u) != 0, kappa, hard, p, q, d);
            } else {
                const int k = t.sup[(int64_t)s * np] - T.n_bool;
                atom_literal(atom_z_state(T, k, st, t.r), T.atom_scale[k], T.atom_strict[k] != 0, kappa, hard, p, q,
                             d);
            }
        }
        W.P(s) = p;
        W.Q(s) = q;
        W.D(s) = d;
    });
    const cptr<Node> nd = T.nodes + t.B.node_off;
    if constexpr (KN > 0) {
        // registers: every iteration up to the bound runs, so no write to the message
        // arrays sits under a branch (a guarded indexed write would make the compiler copy
        // the whole array at the join); iterations past the diagram read a valid node,
        // move no mass and add into the spare entry
#pragma unroll
        for (int v = 0; v < Ms::kArrNodes; ++v) W.M(v) = 0.0f;
        W.M(t.B.root) = 1.0f;
        if (N > 0) {
#pragma unroll
            for (int v = 0; v < KN; ++v) {
                const bool live = v < N;
                const Node x0 = load_node(nd + (live ? v : N - 1));
                const int slot = live ? x0.slot : 0;
                const int hi = live ? x0.hi : Ms::kTrashNode, lo = live ? x0.lo : Ms::kTrashNode;
                const float mv = live ? W.M(v) : 0.0f;
                W.M(hi) += W.P(slot) * mv;
                W.M(lo) += W.Q(slot) * mv;
            }
        }
    } else {
        for_up<0>(0, N + 2, [&](int v) { W.M(v) = 0.0f; });
        W.M(t.B.root) = 1.0f;
        for_up<0>(0, N, [&](int v) {
            const Node x = load_node(nd + v);
            const float mv = W.M(v);
            W.M(x.hi) += W.P(x.slot) * mv;
            W.M(x.lo) += W.Q(x.slot) * mv;
        });
    }
    return t.valid ? W.M(N + 1) : 0.0f;
}

// Reverse pass and chain rule; scatters w * dP[c False]/d(state) through the policy.
template <class Sc, class Ms>
__device__ __forceinline__ void task_backward(const TabView &T, const TaskCtx &t, float wc, const Sc &sc, Ms &W,
                                              int lane) {
    constexpr int KN = Ms::kNodes, KS = Ms::kSlots;
    const int N = t.B.n_nodes, S = t.B.n_slots, NB = t.B.n_bslots;
    const int64_t np = t.B.n_pos;
    const cptr<Node> nd = T.nodes + t.B.node_off;
    if constexpr (KN > 0) {
        // registers: unconditional iterations as in the forward pass; a dead iteration keeps
        // Bm[v] (which may be a terminal) and adds into the spare slot
#pragma unroll
        for (int s = 0; s < Ms::kArrSlots; ++s) W.G(s) = 0.0f;
        W.Bm(N) = 0.0f;
        W.Bm(N + 1) = 1.0f;
        if (N > 0) {
#pragma unroll
            for (int v = KN - 1; v >= 0; --v) {
                const bool live = v < N;
                const Node x0 = load_node(nd + (live ? v : N - 1));
                const int slot = live ? x0.slot : Ms::kTrashSlot;
                const float bh = W.Bm(x0.hi), bl = W.Bm(x0.lo);
                const float bv = W.P(x0.slot) * bh + W.Q(x0.slot) * bl;
                W.Bm(v) = live ? bv : W.Bm(v);
                W.G(slot) += live ? W.M(v) * (bh - bl) : 0.0f;
            }
        }
    } else {
        for_up<0>(0, S, [&](int s) { W.G(s) = 0.0f; });
        W.Bm(N) = 0.0f;
        W.Bm(N + 1) = 1.0f;
        for_down<0>(N, [&](int v) {
            const Node x = load_node(nd + v);
            const float bh = W.Bm(x.hi), bl = W.Bm(x.lo);
            W.Bm(v) = W.P(x.slot) * bh + W.Q(x.slot) * bl;
            W.G(x.slot) += W.M(v) * (bh - bl);
        });
    }
    // Boolean slots: distinct variables within a constraint
    for_up<KS>(0, NB, [&](int s) {
        const float g = t.valid ? wc * W.G(s) * -0.5f : 0.0f;     // dp/da = -1/2
        sc.add_a(t.r, t.valid ? t.sup[(int64_t)s * np] : -1, g, lane);
    });
    if (Ms::kInlineOnly || t.rec) {
        // inline atoms: consecutive atoms on the same variable are summed in registers; a
        // running target is flushed (uniformly across the wave) when the next atom's differs
        int v0 = -1, v1 = -1;
        float g0 = 0.0f, g1 = 0.0f;
        for_up<KS>(NB, S, [&](int s) {
            AtomRec a;
            float gz = 0.0f;
            if (t.valid) {
                a = load_rec(t.rec + (int64_t)(s - NB) * np);
                gz = wc * W.G(s) * W.D(s);
            } else {
                a.v0 = a.v1 = -1;
                a.c0 = a.c1 = 0.0f;
                a.flags = 0;
            }
            const bool n0 = a.v0 != v0, n1 = a.v1 != v1;
            sc.add_b(t.r, n0 ? v0 : -1, n0 ? g0 : 0.0f, lane);
            sc.add_b(t.r, n1 ? v1 : -1, n1 ? g1 : 0.0f, lane);
            if (n0) { v0 = a.v0; g0 = 0.0f; }
            if (n1) { v1 = a.v1; g1 = 0.0f; }
            g0 += gz * a.c0;
            if (a.flags & 2u) g1 += gz * a.c1;
        });
        sc.add_b(t.r, v0, g0, lane);
        sc.add_b(t.r, v1, g1, lane);
    } else if (t.valid) {
        for_up<KS>(NB, S, [&](int s) {
            const float gz = wc * W.G(s) * W.D(s);
            if (gz != 0.0f) {
                const int k = t.sup[(int64_t)s * np] - T.n_bool;
                for (int e = T.atom_ptr[k]; e < T.atom_ptr[k + 1]; ++e)
                    sc.add_b_direct(t.r, T.atom_var[e], gz * (float)T.atom_coef[e]);
            }
        });
    }
}

// ---- pair disjunctions: OR_i (x_{2i} XOR x_{2i+1}) OR a_0 OR ... OR a_{T-1} over the
// Boolean slots 0..2L-1 and the atom slots 2L..2L+T-1 (L in the bucket record). The diagram
// is a chain: one node for x_{2i} and two for x_{2i+1} per pair, then one node per atom; a
// path ends at the false terminal only through the "equal" edges of every pair and the
// "false" edge of every atom. The forward mass of the false terminal is therefore
//   F = prod_i e_i * prod_t q_t,  e_i = p_{2i} p_{2i+1} + q_{2i} q_{2i+1},
// and the reverse sweep's slot sensitivities are F with one factor left out (prefix and
// suffix products): dF/dp_{2i} = (p_{2i+1} - q_{2i+1}) F / e_i, dF/dp_t = -F / q_t.
// Forward and reverse run in one pass with every index known at compile time.
__device__ __forceinline__ float pair_equal(float a0, float a1) {
    const float p0 = (1.0f - a0) * 0.5f, q0 = (1.0f + a0) * 0.5f;
    const float p1 = (1.0f - a1) * 0.5f, q1 = (1.0f + a1) * 0.5f;
    return p0 * p1 + q0 * q1;
}

template <bool kInl, class St>
__device__ __forceinline__ void pair_tail(const TabView &T, const TaskCtx &t, const St &st, int u, double kappa,
                                          bool hard, AtomRec &a, float &q, float &d) {
    const int64_t np = t.B.n_pos;
    float p;
    if (kInl || t.rec) {
        a = load_rec(t.rec + (int64_t)u * np);
        atom_literal(rec_z(a, st, t.r), (double)a.scale, (a.flags & 1u) != 0, kappa, hard, p, q, d);
    } else {
        const int k = t.sup[(int64_t)(t.B.n_bslots + u) * np] - T.n_bool;
        atom_literal(atom_z_state(T, k, st, t.r), T.atom_scale[k], T.atom_strict[k] != 0, kappa, hard, p, q, d);
    }
}

// P[c False] of a pair disjunction (0 for invalid lanes); with kGrad also scatters
// wc * dF/d(state). Every lane reaches the scatter calls (uniform control flow).
template <bool kGrad, bool kInl, class St, class Sc>
__device__ __forceinline__ float pair_eval(const TabView &T, const TaskCtx &t, const St &st, double kappa, bool hard,
                                           float wc, const Sc &sc, int lane) {
    const int L = t.B.pad, NT = t.B.n_slots - 2 * L;
    const int64_t np = t.B.n_pos;
    float e[kPairMaxL], qt[kPairMaxT], dt[kPairMaxT];
    float E = 1.0f, Q = 1.0f;
#pragma unroll
    for (int i = 0; i < kPairMaxL; ++i) {
        e[i] = 1.0f;
        if (i < L && t.valid)
            e[i] = pair_equal(st.av(t.r, t.sup[(int64_t)(2 * i) * np]), st.av(t.r, t.sup[(int64_t)(2 * i + 1) * np]));
        E *= e[i];
    }
#pragma unroll
    for (int u = 0; u < kPairMaxT; ++u) {
        qt[u] = 1.0f;
        dt[u] = 0.0f;
        if (u < NT && t.valid) {
            AtomRec a;
            pair_tail<kInl>(T, t, st, u, kappa, hard, a, qt[u], dt[u]);
        }
        Q *= qt[u];
    }
    const float F = t.valid ? E * Q : 0.0f;
    if constexpr (kGrad) {
        // pairs: rest_i = prod_{j != i} e_j * Q; dF/da_{2i} = rest_i * a_{2i+1} / 2 (dp/da = -1/2)
        float suf[kPairMaxL + 1];
        suf[kPairMaxL] = Q;
#pragma unroll
        for (int i = kPairMaxL - 1; i >= 0; --i) suf[i] = suf[i + 1] * e[i];
        float pre = t.valid ? wc : 0.0f;
#pragma unroll
        for (int i = 0; i < kPairMaxL; ++i) {
            if (i < L) {
                // the pair's values are read again (cached) instead of being kept in registers
                const int i0 = t.valid ? t.sup[(int64_t)(2 * i) * np] : -1;
                const int i1 = t.valid ? t.sup[(int64_t)(2 * i + 1) * np] : -1;
                const float x0 = t.valid ? st.av(t.r, i0) : 0.0f, x1 = t.valid ? st.av(t.r, i1) : 0.0f;
                const float rest = pre * suf[i + 1];
                sc.add_a(t.r, i0, 0.5f * rest * x1, lane);
                sc.add_a(t.r, i1, 0.5f * rest * x0, lane);
            }
            pre *= e[i];
        }
        // atoms: dF/dp_t = -E prod_{t' != t} q_t'; the b-gradient is that times dp/dz and q
        float qs[kPairMaxT + 1];
        qs[kPairMaxT] = 1.0f;
#pragma unroll
        for (int u = kPairMaxT - 1; u >= 0; --u) qs[u] = qs[u + 1] * qt[u];
        float qp = t.valid ? -wc * E : 0.0f;
        if (kInl || t.rec) {
            // consecutive atoms on the same variables are summed before the scatter
            int v0 = -1, v1 = -1;
            float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
            for (int u = 0; u < kPairMaxT; ++u) {
                if (u < NT) {
                    AtomRec a;
                    a.v0 = a.v1 = -1;
                    a.c0 = a.c1 = 0.0f;
                    a.flags = 0;
                    if (t.valid) a = load_rec(t.rec + (int64_t)u * np);
                    const float gz = qp * qs[u + 1] * dt[u];
                    const bool n0 = a.v0 != v0, n1 = a.v1 != v1;
                    sc.add_b(t.r, n0 ? v0 : -1, n0 ? g0 : 0.0f, lane);
                    sc.add_b(t.r, n1 ? v1 : -1, n1 ? g1 : 0.0f, lane);
                    if (n0) { v0 = a.v0; g0 = 0.0f; }
                    if (n1) { v1 = a.v1; g1 = 0.0f; }
                    g0 += gz * a.c0;
                    if (a.flags & 2u) g1 += gz * a.c1;
                }
                qp *= qt[u];
            }
            sc.add_b(t.r, v0, g0, lane);
            sc.add_b(t.r, v1, g1, lane);
        } else {
#pragma unroll
            for (int u = 0; u < kPairMaxT; ++u) {
                const float gz = qp * qs[u + 1] * dt[u];
                if (u < NT && t.valid && gz != 0.0f) {
                    const int k = t.sup[(int64_t)(t.B.n_bslots + u) * np] - T.n_bool;
                    for (int e2 = T.atom_ptr[k]; e2 < T.atom_ptr[k + 1]; ++e2)
                        sc.add_b_direct(t.r, T.atom_var[e2], gz * (float)T.atom_coef[e2]);
                }
                qp *= qt[u];
            }
        }
    }
    return F;
}

// ---- guarded disjunctions (see GdInfo): Boolean selectors 0..k-1 (k <= 2) pick a
// disjunction of literals per assignment g, so the false mass is
//   F = sum_g pi_g prod_{s in S_g} l_s,   l_s = P[literal s False]
// (q_s for a positive literal, p_s for a negated one). The reverse sweep's slot sensitivities
// follow from the same sum: dF/dl_s = sum_{g: s in S_g} pi_g prod_{t in S_g, t != s} l_t
// (prefix and suffix products, no division), and for a selector dF/dp_i = sum_g (+-1)
// (pi_g / P[slot i = g_i]) prod_g. Boolean and atom slots sit in register arrays with static
// indices; the masks and run flags are wave-uniform (one scalar record per template). Every
// lane issues all of its table reads up front (lanes on padding positions or past the
// restarts read position and restart 0, which exist), so their latencies overlap.
__device__ __forceinline__ GdInfo load_gd(cptr<GdInfo> p) {
    static_assert(sizeof(GdInfo) == 64, "guarded-disjunction record layout");
    typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
    const i32x16 raw = *(cptr<i32x16>)p;
    GdInfo g;
    __builtin_memcpy(&g, &raw, sizeof(g));
    return g;
}

// Literal probability of an atom from q.b already formed (lin), as atom_literal but with the
// derivative's scale in FP32: p = erfc(u)/2, u = kappa scale (lin - rhs) (FP64 product,
// rounded once), dp/dz = -kappa scale/sqrt(pi) e^{-u^2}.
__device__ __forceinline__ void gd_atom(double lin, float rhs, float scale, bool strict, double kappa, bool hard,
                                        float &p, float &q, float &d) {
#pragma clang fp contract(off)
    const double z = lin - (double)rhs;
    if (hard) {
        const bool tr = strict ? (z < 0.0) : (z <= 0.0);
        p = tr ? 1.0f : 0.0f;
        q = tr ? 0.0f : 1.0f;
        d = 0.0f;
    } else {
        const double ks = kappa * (double)scale;
        const float u = (float)(z * ks);
        float emu2;
        // the smaller of p, 1-p; a NaN u gives a NaN e (rcp, exp2 and fma keep NaN), so p
        // and q are NaN too
        const float e = 0.5f * erfc_nr(fabsf(u), emu2);
        p = (u >= 0.0f) ? e : 1.0f - e;
        q = (u >= 0.0f) ? 1.0f - e : e;
        d = -((float)ks * 0.56418958354775628695f) * emu2;
    }
}

__device__ __forceinline__ SlimRec load_slim(cptr<SlimRec> p) {
    const cptr<int32_t> q = (cptr<int32_t>)p;
    return SlimRec{q[0], q[1], __int_as_float(q[2])};
}

// kSlim: the atoms come from the slim records and the template's form (the per-call
// kernel, where the table stream is the cost); otherwise from the 32-byte records, which
// keep the form out of the scalar registers of the fused solver's kernels.
template <int NBm, int NAm, bool kGrad, bool kSlim, class St, class Sc>
__device__ __forceinline__ float gd_eval_n(const TabView &T, const TaskCtx &t, const GdInfo &g, const St &st,
                                           double kappa, bool hard, float wc, const Sc &sc, int lane) {
    const int NB = t.B.n_bslots, NA = t.B.n_slots - t.B.n_bslots, k = g.k;
    const int64_t np = t.B.n_pos;
    const int rr = t.valid ? t.r : 0;   // a row that exists for the reads of invalid lanes
    // the template's per-slot coefficients, scales and flags (wave-uniform, scalar loads)
    const cptr<GdForm> form = T.gdf + t.B.tpl;
    // ---- reads: Boolean ids and slim atom records (slots past the template's count re-read
    // its last one, so no read depends on a per-slot branch), then the state values they name
    const int S = NB + NA;
    int idb[NBm];
#pragma unroll
    for (int i = 0; i < NBm; ++i) idb[i] = t.sup[(int64_t)(i < S ? i : S - 1) * np];
    using Rec = typename std::conditional<kSlim, SlimRec, AtomRec>::type;
    Rec rec[NAm];
    if (NA > 0) {
        if constexpr (kSlim) {
            const cptr<SlimRec> sp = T.srec + form->srec_base + t.local;
#pragma unroll
            for (int j = 0; j < NAm; ++j) rec[j] = load_slim(sp + (int64_t)(j < NA ? j : NA - 1) * np);
        } else {
#pragma unroll
            for (int j = 0; j < NAm; ++j) rec[j] = load_rec(t.rec + (int64_t)(j < NA ? j : NA - 1) * np);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NAm; ++j) rec[j] = Rec{};
    }
    float av[NBm], y0[NAm], y1[NAm];
#pragma unroll
    for (int i = 0; i < NBm; ++i) av[i] = st.av(rr, i < NB ? idb[i] : 0);
#pragma unroll
    for (int j = 0; j < NAm; ++j) {
        // a run of atoms on the same variables reads their values once
        const bool same = j > 0 && ((g.same_vars >> j) & 1u);
        y0[j] = same ? y0[j - 1] : st.bv(rr, rec[j].v0);
        y1[j] = same ? y1[j - 1] : st.bv(rr, rec[j].v1);   // v1 = v0 for one-variable atoms
    }
    // Booleans: P[True] = (1 - a)/2; literal-false probabilities l (negated literal: P[True])
    float pb[NBm], qb[NBm], lb[NBm];
#pragma unroll
    for (int i = 0; i < NBm; ++i) {
        pb[i] = (1.0f - av[i]) * 0.5f;
        qb[i] = (1.0f + av[i]) * 0.5f;
        lb[i] = ((g.neg >> i) & 1u) ? pb[i] : qb[i];
    }
    // atoms: q.b in FP64 in the stored multiply-then-add order, once per run of equal forms;
    // only the coefficients (for the scatter), l and dp/dz stay live past this loop
    const uint32_t negA = g.neg >> NB;
    float la[NAm], da[NAm], c0[NAm], c1[NAm];
    {
        double lin = 0.0;
#pragma unroll
        for (int j = 0; j < NAm; ++j) {
            float scale;
            bool two, strict;
            if constexpr (kSlim) {
                const uint32_t fl = form->flags;
                c0[j] = form->c0[j];   // slots past the template's count hold 0
                c1[j] = form->c1[j];   // 0 for one-variable atoms
                scale = form->scale[j];
                two = (fl >> (8 + j)) & 1u;
                strict = (fl >> j) & 1u;
            } else {
                c0[j] = rec[j].c0;
                c1[j] = rec[j].c1;
                scale = rec[j].scale;
                two = (rec[j].flags & 2u) != 0;
                strict = (rec[j].flags & 1u) != 0;
            }
            if (j == 0 || !((g.same_lin >> j) & 1u)) {
#pragma clang fp contract(off)
                double acc = (double)c0[j] * (double)y0[j];   // the stored first product
                if (two) {
                    const double p1 = (double)c1[j] * (double)y1[j];
                    acc = acc + p1;
                }
                lin = acc;
            }
            float pj, qj;
            gd_atom(lin, rec[j].rhs, scale, strict, kappa, hard, pj, qj, da[j]);
            la[j] = ((negA >> j) & 1u) ? pj : qj;
        }
    }
    // ---- sum over the selector assignments
    float F = 0.0f, gp0 = 0.0f, gp1 = 0.0f;
    float glb[NBm], gla[NAm];
#pragma unroll
    for (int i = 0; i < NBm; ++i) glb[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < NAm; ++j) gla[j] = 0.0f;
    if constexpr (NBm >= 2) {
        if (g.sep) {   // the product of the two selectors' sums (see GdInfo::sep)
            static_assert(NAm == kGdMaxAtoms, "sep_slots name a missing atom kGdMaxAtoms: lx[NAm] holds its 1");
            float lx[NAm + 1], L[8];
#pragma unroll
            for (int j = 0; j < NAm; ++j) lx[j] = la[j];
            lx[NAm] = 1.0f;
#pragma unroll
            for (int i = 0; i < 8; ++i) L[i] = lx[(g.sep_slots >> (4 * i)) & 15u];
            const float P00 = L[0] * L[1], P01 = L[2] * L[3], P10 = L[4] * L[5], P11 = L[6] * L[7];
            const float SA = qb[0] * P00 + pb[0] * P01, SB = qb[1] * P10 + pb[1] * P11;
            F = SA * SB;
            if constexpr (kGrad) {
                gp0 = (P01 - P00) * SB;
                gp1 = (P11 - P10) * SA;
                const float wq[4] = {qb[0] * SB, pb[0] * SB, qb[1] * SA, pb[1] * SA};
                float gx[NAm + 1];
#pragma unroll
                for (int j = 0; j <= NAm; ++j) gx[j] = 0.0f;
#pragma unroll
                for (int i = 0; i < 8; ++i) gx[(g.sep_slots >> (4 * i)) & 15u] = wq[i >> 1] * L[i ^ 1];
#pragma unroll
                for (int j = 0; j < NAm; ++j) gla[j] = gx[j];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < (1 << kGdMaxSel); ++c) {
        if (g.sep) break;
        if (c >= (1 << k)) break;
        const uint32_t m = g.mask[c];
        if (m >> 31) continue;   // this assignment reaches the True terminal
        const uint32_t mA = m >> NB;
        // selectors are Boolean slots (k <= NB <= NBm)
        const float pi0 = k > 0 ? ((c & 1) ? pb[0] : qb[0]) : 1.0f;
        float pi1 = 1.0f;
        if constexpr (NBm > 1) {
            if (k > 1) pi1 = (c & 2) ? pb[1] : qb[1];
        }
        // factors: l where the slot is in the disjunction, else 1
        float fb[NBm], fa[NAm], preb[NBm], prea[NAm];
        float prod = 1.0f;
#pragma unroll
        for (int i = 0; i < NBm; ++i) {
            fb[i] = (i < NB && ((m >> i) & 1u)) ? lb[i] : 1.0f;
            preb[i] = prod;
            prod *= fb[i];
        }
#pragma unroll
        for (int j = 0; j < NAm; ++j) {
            fa[j] = (j < NA && ((mA >> j) & 1u)) ? la[j] : 1.0f;
            prea[j] = prod;
            prod *= fa[j];
        }
        F += (pi0 * pi1) * prod;
        if constexpr (kGrad) {
            float suf = pi0 * pi1;
#pragma unroll
            for (int j = NAm - 1; j >= 0; --j) {
                if (j < NA && ((mA >> j) & 1u)) gla[j] += prea[j] * suf;
                suf *= fa[j];
            }
#pragma unroll
            for (int i = NBm - 1; i >= 0; --i) {
                if (i < NB && ((m >> i) & 1u)) glb[i] += preb[i] * suf;
                suf *= fb[i];
            }
            if (k > 0) gp0 += ((c & 1) ? pi1 : -pi1) * prod;
            if (k > 1) gp1 += ((c & 2) ? pi0 : -pi0) * prod;
        }
    }
    if constexpr (kGrad) {
        const float wv = t.valid ? wc : 0.0f;
        // Boolean slots (distinct variables): G = dF/dp (a negated literal's l is p, a
        // positive one's 1 - p; a selector's from the sum above), dp/da = -1/2
#pragma unroll
        for (int i = 0; i < NBm; ++i) {
            if (i < NB) {
                float G = ((g.neg >> i) & 1u) ? glb[i] : -glb[i];
                if (i == 0 && k > 0) G = gp0;
                if (i == 1 && k > 1) G = gp1;
                sc.add_a(t.r, t.valid ? idb[i] : -1, wv * G * -0.5f, lane);
            }
        }
        // atoms: dz = w dF/dp dp/dz, summed over a run of atoms on the same variables and
        // scattered at the run's end
        float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
        for (int j = 0; j < NAm; ++j) {
            if (j < NA) {
                const float G = ((negA >> j) & 1u) ? gla[j] : -gla[j];
                const float gz = wv * G * da[j];
                g0 += gz * c0[j];
                g1 += gz * c1[j];
                const bool last = j + 1 >= NA || !((g.same_vars >> (j + 1)) & 1u);
                if (last) {
                    sc.add_b(t.r, t.valid ? rec[j].v0 : -1, g0, lane);
                    sc.add_b(t.r, t.valid ? rec[j].v1 : -1, g1, lane);   // g1 = 0 for one variable
                    g0 = g1 = 0.0f;
                }
            }
        }
    }
    return t.valid ? F : 0.0f;
}

// Message-store variants: a kernel is instantiated per variant and the host picks the
// smallest whose bounds hold for every diagram of the launch.
enum MsgVariant { kMsgLds = 0, kMsgSmall = 1, kMsgMedium = 2, kMsgLarge = 3 };
template <int V> struct MsgOf;
template <> struct MsgOf<kMsgSmall> { using type = RegMsgs<4, 4>; };
template <> struct MsgOf<kMsgMedium> { using type = RegMsgs<20, 12>; };
template <> struct MsgOf<kMsgLarge> { using type = RegMsgs<kLargeMaxNodes, kLargeMaxSlots>; };
template <> struct MsgOf<kMsgLds> { using type = LdsMsgs; };

// Bind a store: an LDS store to the wave's columns (base: this wave's LDS scratch), a
// register store to the kernel's local arrays.
template <class Ms>
__device__ __forceinline__ void bind_msgs(Ms &W, float *base, int NN, int SS, int lane, float *m, float *b, float *p,
                                          float *q, float *d, float *g) {
    if constexpr (Ms::kNodes == 0) {
        W.W = WaveScratch::at(base, NN, SS);
        W.lane = lane;
    } else {
        W.m_ = m;
        W.b_ = b;
        W.p_ = p;
        W.q_ = q;
        W.d_ = d;
        W.g_ = g;
    }
}
// Declares the store W of type Ms with its register arrays (unused for LDS stores).
#define FSMT_MSG_STORE(Ms, W, base, NN, SS, lane)                                                              \
    float W##_m[Ms::kArrNodes], W##_b[Ms::kArrNodes], W##_p[Ms::kArrSlots], W##_q[Ms::kArrSlots],               \
        W##_d[Ms::kArrSlots], W##_g[Ms::kArrSlots];                                                             \
    Ms W;                                                                                                       \
    bind_msgs(W, base, NN, SS, lane, W##_m, W##_b, W##_p, W##_q, W##_d, W##_g)

// One (constraint, restart) task: P[c False], and with kGrad the reverse sweep's gradient
// scattered through the policy. With kCF > 0 a register message store is declared per task,
// so its arrays are live only in the generic branch.
template <bool kGrad, int kCF, bool kSlim = false, class St, class Sc, class Ms>
__device__ __forceinline__ float task_eval(const TabView &T, const TaskCtx &t, const St &st, double kappa, bool hard,
                                           float wc, const Sc &sc, Ms &W, int lane) {
    if constexpr (kCF > 0) {
        if constexpr (kCF >= 3) {
            if (t.B.pad > 0) return pair_eval<kGrad, Ms::kInlineOnly>(T, t, st, kappa, hard, wc, sc, lane);
        }
        if (t.B.pad < 0) {
            const GdInfo g = load_gd(T.gd + t.B.tpl);
            const int NB = t.B.n_bslots, NA = t.B.n_slots - t.B.n_bslots;
            if (NB <= 1 && NA <= 2) return gd_eval_n<1, 2, kGrad, kSlim>(T, t, g, st, kappa, hard, wc, sc, lane);
            if constexpr (kCF >= 2) {
                if (NB <= 2) return gd_eval_n<2, kGdMaxAtoms, kGrad, kSlim>(T, t, g, st, kappa, hard, wc, sc, lane);
            }
            if constexpr (kCF >= 3) return gd_eval_n<kGdMaxBool, kGdMaxAtoms, kGrad, kSlim>(T, t, g, st, kappa, hard, wc, sc, lane);
        }
        if constexpr (Ms::kNodes > 0) {
            FSMT_MSG_STORE(Ms, Wt, nullptr, 0, 0, lane);
            const float unsat = task_forward(T, t, st, kappa, hard, Wt);
            if constexpr (kGrad) task_backward(T, t, wc, sc, Wt, lane);
            return unsat;
        }
    }
    const float unsat = task_forward(T, t, st, kappa, hard, W);
    if constexpr (kGrad) task_backward(T, t, wc, sc, W, lane);
    return unsat;
}

// The LDS store is used when asked for, and for instances with pair-disjunction templates:
// their kernels carry the closed-form path beside the generic one, and the generic
// templates in LDS leave it the registers (scheduling 256 x 5: 4.2 ms per PGD step against
// 5.4 ms with register stores; placement 64 x 8: 1.69 against 1.62 ms).
inline bool lds_store(const fsmt_xbdd *h) {
    return h->lds_messages || ((h->n_pair > 0 || h->n_gd > 0) && h->small_max_nodes > 0);
}
// Closed-form level an instance needs (see gd_level_of; 0 when it has no closed-form template).
inline int closed_level(const fsmt_xbdd *h) { return h->n_pair > 0 ? 3 : h->gd_level; }

// Register variants need every atom in an inline record (the CSR path is compiled out).
inline int msg_variant(int max_nodes, int max_slots, bool lds_only, bool all_inline) {
    if (lds_only || !all_inline) return kMsgLds;
    if (max_nodes <= 4 && max_slots <= 4) return kMsgSmall;
    if (max_nodes <= 20 && max_slots <= 12) return kMsgMedium;
    if (max_nodes <= kLargeMaxNodes && max_slots <= kLargeMaxSlots) return kMsgLarge;
    return kMsgLds;
}

// ---- big diagrams: level-synchronous evaluation of one (constraint, restart) by a wave
// Nodes are stored level by level (sorted by slot), so a level is a contiguous range; its
// nodes go to the lanes, and lanes also take the slots for the literal probabilities and
// the scatter. The wave's LDS rows hold the constraint's node table and the messages: M and
// Bm per node, P, Q, D, G per slot.
//   forward : per level, each node adds p M[v] to M[hi] and (1-p) M[v] to M[lo] (LDS
//             atomics: nodes of one level may share children, which lie on deeper levels)
//   reverse : per level from the bottom, Bm[v] = p Bm[hi] + (1-p) Bm[lo] (children final),
//             and the level's sensitivity G[s] = sum_v M[v] (Bm[hi] - Bm[lo]) is a wave sum
// One wavefront per constraint: only LDS waits order the levels, no barrier.
// Restarts per wavefront task: each task stages the node table once for its chunk; small
// chunks give more parallel waves when there are few big constraints.
inline int level_chunk(int64_t n_big_restarts, int n_cu) {
    const int64_t target = (int64_t)n_cu * 16;   // about four waves per SIMD
    int chunk = 1;
    while (chunk < 8 && n_big_restarts / (2 * chunk) >= target) chunk *= 2;
    return chunk;
}

// floats of one wave's LDS rows: node table (2 words a node), M, Bm, P, Q, D, G
__host__ __device__ inline size_t level_wave_floats(int max_nodes, int max_slots) {
    return (size_t)2 * max_nodes + 2 * ((size_t)max_nodes + 2) + 4 * (size_t)max_slots;
}

struct LevelRows {
    uint2 *NL;
    float *M, *Bm, *P, *Q, *D, *G;
    __device__ __forceinline__ static LevelRows at(float *base, int max_nodes, int max_slots) {
        LevelRows w;
        w.NL = reinterpret_cast<uint2 *>(base);
        w.M = base + 2 * max_nodes;
        w.Bm = w.M + max_nodes + 2;
        w.P = w.Bm + max_nodes + 2;
        w.Q = w.P + max_slots;
        w.D = w.Q + max_slots;
        w.G = w.D + max_slots;
        return w;
    }
};

struct LevelCtx {
    BucketInfo B;
    int c, local;
    cptr<int32_t> sup, lev;
    cptr<AtomRec> rec;
};

__device__ __forceinline__ LevelCtx level_ctx(const TabView &T, cptr<int32_t> lev_all, int pos_in) {
    LevelCtx L;
    const int pos = __builtin_amdgcn_readfirstlane(pos_in);
    L.B = load_bucket(T.bucket + __builtin_amdgcn_readfirstlane(T.task_bucket[pos >> 6]));
    L.c = __builtin_amdgcn_readfirstlane(T.pos_con[pos]);
    L.local = pos - L.B.pos_begin;
    L.sup = T.sup + L.B.sup_base + L.local;
    L.rec = L.B.arec_base >= 0 ? T.arec + L.B.arec_base + L.local : nullptr;
    L.lev = lev_all + L.B.lev_off;
    return L;
}

// Objective partial sums of one wave for a block of consecutive restarts (lane i holds
// restart base + i, at most 64): added to the accumulators with one atomic per restart when
// the wave moves to another block and at the end. One float atomic per (constraint,
// restart) into a large sum would round away a bias when many constraints add the same
// value; per-wave partial sums keep the number of such additions small.
struct WaveObjAcc {
    float *obj;
    int base = -1, count = 0;
    float acc = 0.0f;
    __device__ __forceinline__ void flush(int lane) {
        if (obj && base >= 0 && lane < count && acc != 0.0f) atomic_add_f32(obj + base + lane, acc);
        acc = 0.0f;
    }
    __device__ __forceinline__ void begin(int b, int n, int lane) {
        if (b != base || n != count) {
            flush(lane);
            base = b;
            count = n;
        }
    }
    __device__ __forceinline__ void add(int i, float v, int lane) {
        if (lane == i) acc += v;
    }
};

__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ Node unpack_node(uint2 raw) {
    Node n;
    n.slot = (uint16_t)(raw.x & 0xFFFFu);
    n.hi = (uint16_t)(raw.x >> 16);
    n.lo = (uint16_t)(raw.y & 0xFFFFu);
    n.pad = 0;
    return n;
}

// Copy the constraint's node table into the wave's LDS rows.
__device__ __forceinline__ void level_stage_nodes(const TabView &T, const LevelCtx &L, const LevelRows &W, int lane) {
    wave_lds_sync();   // the previous task's readers are done
    const cptr<u32x2> nd = (cptr<u32x2>)(T.nodes + L.B.node_off);
    for (int v = lane; v < L.B.n_nodes; v += 64) {
        const u32x2 raw = nd[v];
        W.NL[v] = make_uint2(raw.x, raw.y);
    }
    wave_lds_sync();
}

// Forward (and with grad the reverse pass and the scatter of wc * dP[c False]/d(state))
// for restart r; returns P[c False] in every lane.
template <class St, class Sc>
__device__ __forceinline__ float level_eval(const TabView &T, const LevelCtx &L, const St &st, const Sc &sc, int r,
                                            double kappa, bool hard, float wc, bool grad, const LevelRows &W,
                                            int lane) {
    const int N = L.B.n_nodes, S = L.B.n_slots, NB = L.B.n_bslots;
    const int64_t np = L.B.n_pos;
    // with fewer than 64 slots, lane s keeps slot s's probabilities and level start s in
    // registers and the level loops read them with v_readlane instead of memory loads
    const bool in_regs = S < 64;
    float p_lane = 0.0f, q_lane = 0.0f;
    int lev_lane = 0;
    if (in_regs && lane <= S) lev_lane = L.lev[lane];
    for (int s = lane; s < S; s += 64) {
        float p, qq, d = 0.0f;
        if (s < NB) {
            const float av = st.av(r, L.sup[(int64_t)s * np]);
            p = (1.0f - av) * 0.5f;
            qq = (1.0f + av) * 0.5f;
        } else if (L.rec) {
            const AtomRec at = load_rec(L.rec + (int64_t)(s - NB) * np);
            atom_literal(rec_z(at, st, r), (double)at.scale, (at.flags & 1u) != 0, kappa, hard, p, qq, d);
        } else {
            const int k = L.sup[(int64_t)s * np] - T.n_bool;
            atom_literal(atom_z_state(T, k, st, r), T.atom_scale[k], T.atom_strict[k] != 0, kappa, hard, p, qq, d);
        }
        W.P[s] = p;
        W.Q[s] = qq;
        W.D[s] = d;
        p_lane = p;
        q_lane = qq;
    }
    auto level_of = [&](int s, int &v0, int &v1, float &p, float &qq) {
        if (in_regs) {
            v0 = __builtin_amdgcn_readlane(lev_lane, s);
            v1 = __builtin_amdgcn_readlane(lev_lane, s + 1);
            p = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p_lane), s));
            qq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q_lane), s));
        } else {
            v0 = L.lev[s];
            v1 = L.lev[s + 1];
            p = W.P[s];
            qq = W.Q[s];
        }
    };
    for (int v = lane; v < N + 2; v += 64) W.M[v] = 0.0f;
    wave_lds_sync();
    if (lane == 0) W.M[L.B.root] = 1.0f;
    wave_lds_sync();
    for (int s = 0; s < S; ++s) {
        int v0, v1;
        float p, qq;
        level_of(s, v0, v1, p, qq);
        if (v0 == v1) continue;
        for (int v = v0 + lane; v < v1; v += 64) {
            const Node x = unpack_node(W.NL[v]);
            const float mv = W.M[v];
            atomicAdd(W.M + x.hi, p * mv);
            atomicAdd(W.M + x.lo, qq * mv);
        }
        wave_lds_sync();
    }
    const float unsat = W.M[N + 1];
    if (grad) {
        if (lane == 0) {
            W.Bm[N] = 0.0f;
            W.Bm[N + 1] = 1.0f;
        }
        wave_lds_sync();
        for (int s = S - 1; s >= 0; --s) {
            int v0, v1;
            float p, qq;
            level_of(s, v0, v1, p, qq);
            float g = 0.0f;
            if (v0 < v1) {
                for (int v = v0 + lane; v < v1; v += 64) {
                    const Node x = unpack_node(W.NL[v]);
                    const float bh = W.Bm[x.hi], bl = W.Bm[x.lo];
                    W.Bm[v] = p * bh + qq * bl;
                    g += W.M[v] * (bh - bl);
                }
                g = wave_sum(g);
            }
            if (lane == 0) W.G[s] = g;
            wave_lds_sync();
        }
        for (int s = lane; s < S; s += 64) {
            const float g = wc * W.G[s];
            if (s < NB) {
                sc.add_a_direct(r, L.sup[(int64_t)s * np], g * -0.5f);   // dp/da = -1/2
            } else if (L.rec) {
                const AtomRec at = load_rec(L.rec + (int64_t)(s - NB) * np);
                const float gz = g * W.D[s];
                if (gz != 0.0f) {
                    sc.add_b_direct(r, at.v0, gz * at.c0);
                    if (at.flags & 2u) sc.add_b_direct(r, at.v1, gz * at.c1);
                }
            } else {
                const float gz = g * W.D[s];
                if (gz != 0.0f) {
                    const int k = L.sup[(int64_t)s * np] - T.n_bool;
                    for (int e = T.atom_ptr[k]; e < T.atom_ptr[k + 1]; ++e)
                        sc.add_b_direct(r, T.atom_var[e], gz * (float)T.atom_coef[e]);
                }
            }
        }
    }
    wave_lds_sync();   // the next restart overwrites the message rows
    return unsat;
}

// Deterministic walk of constraint c at the rounded point (exact check).
template <class St>
__device__ __forceinline__ bool walk_state(const TabView &T, const St &st, int c, int r) {
    const BucketInfo B = load_bucket(T.bucket + T.con_bucket[c]);
    const int local = T.con_local[c];
    const cptr<int32_t> s = T.sup + B.sup_base + local;
    const int N = B.n_nodes;
    int v = B.root;
    while (v < N) {
        const Node x = load_node_lane(T.nodes + B.node_off + v);   // each lane walks its own diagram
        bool tr;
        if (x.slot < B.n_bslots) {
            tr = st.av(r, s[(int64_t)x.slot * B.n_pos]) < 0.0f;
        } else if (B.arec_base >= 0) {
            const AtomRec a = load_rec(T.arec + B.arec_base + (int64_t)(x.slot - B.n_bslots) * B.n_pos + local);
            const double z = rec_z(a, st, r);
            tr = (a.flags & 1u) ? (z < 0.0) : (z <= 0.0);
        } else {
            const int k = s[(int64_t)x.slot * B.n_pos] - T.n_bool;
            const double z = atom_z_state(T, k, st, r);
            tr = T.atom_strict[k] ? (z < 0.0) : (z <= 0.0);
        }
        v = tr ? x.hi : x.lo;
    }
    return v == N;
}

}  // namespace fsmt
