// One wavefront task of the diagram passes, shared by the per-call kernel and the fused
// solver. A task is 64 lanes, each a (constraint position, restart) pair of one bucket, so
// the diagram shape is uniform across the wave: node records come through the scalar unit
// and each lane keeps its messages in its own LDS column ([row][lane] layout).
//
// State access and gradient accumulation are template policies: global strided views with
// L2 atomics (per-call path) or LDS-resident state with LDS atomics (fused solver).
#pragma once
#include "kernels_common.hpp"

namespace fsmt {

// Device pointers of one compiled instance.
struct TabView {
    const TplInfo *tpl;
    const Node *nodes;
    const BucketInfo *bucket;
    const int32_t *bucket_start;
    const int32_t *pos_con;
    const int32_t *sup;
    const int32_t *con_bucket;
    const int32_t *con_local;
    const int32_t *atom_ptr;
    const int32_t *atom_var;
    const double *atom_coef;
    const double *atom_rhs;
    const double *atom_scale;
    const uint8_t *atom_strict;
    const float *real_lo;
    const float *real_hi;
    int32_t n_bool, n_real, n_cons, n_pos, n_buckets, pad;

    static TabView of(const fsmt_xbdd *h) {
        TabView t;
        t.tpl = h->d.tpl;
        t.nodes = h->d.nodes;
        t.bucket = h->d.bucket;
        t.bucket_start = h->d.bucket_start;
        t.pos_con = h->d.pos_con;
        t.sup = h->d.sup;
        t.con_bucket = h->d.con_bucket;
        t.con_local = h->d.con_local;
        t.atom_ptr = h->d.atom_ptr;
        t.atom_var = h->d.atom_var;
        t.atom_coef = h->d.atom_coef;
        t.atom_rhs = h->d.atom_rhs;
        t.atom_scale = h->d.atom_scale;
        t.atom_strict = h->d.atom_strict;
        t.real_lo = h->d.real_lo;
        t.real_hi = h->d.real_hi;
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
struct GlobalScatter {
    View ga, gb;
    __device__ __forceinline__ void add_a(int r, int i, float g) const { atomic_add_f32(&ga.at(r, i), g); }
    __device__ __forceinline__ void add_b(int r, int j, float g) const { atomic_add_f32(&gb.at(r, j), g); }
};
struct LdsScatter {
    float *ga, *gb;
    __device__ __forceinline__ void add_a(int, int i, float g) const { atomicAdd(ga + i, g); }
    __device__ __forceinline__ void add_b(int, int j, float g) const { atomicAdd(gb + j, g); }
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

// Find the bucket containing position pos (uniform across the wave).
__device__ __forceinline__ int find_bucket(const int32_t *start, int nb, int pos) {
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
    BucketInfo B;
    TplInfo Tp;
    const int32_t *sup;   // this lane's support column
    int c;                // original constraint id (or -1)
    int r;
    bool valid;
};

// Locate the task: pos is this lane's position, all lanes of the wave in one bucket.
__device__ __forceinline__ TaskCtx task_ctx(const TabView &T, int pos, int r, bool r_ok) {
    TaskCtx t;
    const int pos0 = __builtin_amdgcn_readfirstlane(pos);
    const int bk = find_bucket(T.bucket_start, T.n_buckets, pos0);
    t.B = T.bucket[bk];
    t.Tp = T.tpl[t.B.tpl];
    t.sup = T.sup + t.B.sup_base + (pos - t.B.pos_begin);
    t.c = T.pos_con[pos];
    t.r = r;
    t.valid = (t.c >= 0) && r_ok;
    return t;
}

// Literal probabilities and the forward pass; returns P[c False] (0 for invalid lanes).
template <class St>
__device__ __forceinline__ float task_forward(const TabView &T, const TaskCtx &t, const St &st, double kappa,
                                              bool hard, const WaveScratch &W, int lane) {
    const int N = t.Tp.n_nodes, S = t.Tp.n_slots, NB = t.Tp.n_bslots;
    const int64_t np = t.B.n_pos;
    for (int s = 0; s < NB; ++s) {
        const float av = t.valid ? st.av(t.r, t.sup[(int64_t)s * np]) : 0.0f;
        W.P[s * 64 + lane] = (1.0f - av) * 0.5f;
        W.Q[s * 64 + lane] = (1.0f + av) * 0.5f;
    }
    for (int s = NB; s < S; ++s) {
        float p = 0.5f, q = 0.5f, d = 0.0f;
        if (t.valid) {
            const int k = t.sup[(int64_t)s * np] - T.n_bool;
            const double z = atom_z_state(T, k, st, t.r);
            if (hard) {
                const bool tr = T.atom_strict[k] ? (z < 0.0) : (z <= 0.0);
                p = tr ? 1.0f : 0.0f;
                q = tr ? 0.0f : 1.0f;
            } else {
                const double ks = kappa * T.atom_scale[k];
                const float u = (float)(z * ks);
                const float e = 0.5f * erfcf(fabsf(u));          // the smaller of p, 1-p
                p = (u >= 0.0f) ? e : 1.0f - e;
                q = (u >= 0.0f) ? 1.0f - e : e;
                if (u != u) { p = u; q = u; }                    // NaN in, NaN out
                d = -(float)(ks * 0.56418958354775628695) * expf(-u * u);   // dp/dz = -k s/sqrt(pi) e^-u^2
            }
        }
        W.P[s * 64 + lane] = p;
        W.Q[s * 64 + lane] = q;
        W.D[s * 64 + lane] = d;
    }
    for (int v = 0; v < N + 2; ++v) W.M[v * 64 + lane] = 0.0f;
    W.M[t.Tp.root * 64 + lane] = 1.0f;
    const Node *nd = T.nodes + t.Tp.node_off;
    for (int v = 0; v < N; ++v) {
        const Node x = load_node(nd + v);
        const float mv = W.M[v * 64 + lane];
        W.M[x.hi * 64 + lane] += W.P[x.slot * 64 + lane] * mv;
        W.M[x.lo * 64 + lane] += W.Q[x.slot * 64 + lane] * mv;
    }
    return t.valid ? W.M[(N + 1) * 64 + lane] : 0.0f;
}

// Reverse pass and chain rule; scatters w * dP[c False]/d(state) through the policy.
template <class Sc>
__device__ __forceinline__ void task_backward(const TabView &T, const TaskCtx &t, float wc, const Sc &sc,
                                              const WaveScratch &W, int lane) {
    const int N = t.Tp.n_nodes, S = t.Tp.n_slots, NB = t.Tp.n_bslots;
    const int64_t np = t.B.n_pos;
    for (int s = 0; s < S; ++s) W.G[s * 64 + lane] = 0.0f;
    W.Bm[N * 64 + lane] = 0.0f;
    W.Bm[(N + 1) * 64 + lane] = 1.0f;
    const Node *nd = T.nodes + t.Tp.node_off;
    for (int v = N - 1; v >= 0; --v) {
        const Node x = load_node(nd + v);
        const float bh = W.Bm[x.hi * 64 + lane], bl = W.Bm[x.lo * 64 + lane];
        W.Bm[v * 64 + lane] = W.P[x.slot * 64 + lane] * bh + W.Q[x.slot * 64 + lane] * bl;
        W.G[x.slot * 64 + lane] += W.M[v * 64 + lane] * (bh - bl);
    }
    if (!t.valid) return;
    for (int s = 0; s < NB; ++s) {
        const float g = wc * W.G[s * 64 + lane] * -0.5f;     // dp/da = -1/2
        if (g != 0.0f) sc.add_a(t.r, t.sup[(int64_t)s * np], g);
    }
    for (int s = NB; s < S; ++s) {
        const float gz = wc * W.G[s * 64 + lane] * W.D[s * 64 + lane];
        if (gz == 0.0f) continue;
        const int k = t.sup[(int64_t)s * np] - T.n_bool;
        for (int e = T.atom_ptr[k]; e < T.atom_ptr[k + 1]; ++e) sc.add_b(t.r, T.atom_var[e], gz * (float)T.atom_coef[e]);
    }
}

// Deterministic walk of constraint c at the rounded point (exact check).
template <class St>
__device__ __forceinline__ bool walk_state(const TabView &T, const St &st, int c, int r) {
    const BucketInfo B = T.bucket[T.con_bucket[c]];
    const TplInfo Tp = T.tpl[B.tpl];
    const int32_t *s = T.sup + B.sup_base + T.con_local[c];
    const int N = Tp.n_nodes;
    int v = Tp.root;
    while (v < N) {
        const Node x = T.nodes[Tp.node_off + v];
        const int id = s[(int64_t)x.slot * B.n_pos];
        bool tr;
        if (x.slot < Tp.n_bslots) {
            tr = st.av(r, id) < 0.0f;
        } else {
            const int k = id - T.n_bool;
            const double z = atom_z_state(T, k, st, r);
            tr = T.atom_strict[k] ? (z < 0.0) : (z <= 0.0);
        }
        v = tr ? x.hi : x.lo;
    }
    return v == N;
}

}  // namespace fsmt
