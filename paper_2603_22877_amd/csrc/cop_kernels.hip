// HIP kernels for gfx950 (CDNA4, wave64) and the per-call C ABI entry points:
// cop_forward, cop_backward, pgd_step, round_and_check.
//
// Work decomposition of the diagram passes. A "task" is one wavefront's worth of
// (constraint, restart) pairs. With R_pad = next power of two >= R (R <= 64) a task covers
// 64/R_pad consecutive constraint positions times R_pad restarts (lane = position-major,
// restart-minor); with R > 64 a task is one position times 64 restarts. Buckets are padded
// to 64 positions, so every lane of a wave walks the same diagram shape: node records are
// wave-uniform and are fetched through the scalar unit (s_load), while each lane keeps its
// own messages in an LDS column ([node][lane] layout, conflict-free, indexed by the
// uniform node id). Probabilities are evaluated once per (slot, lane) before the passes.
//
// Per (constraint c, restart r) the kernel computes (paper, Supplementary Note 5):
//   forward  : m_td[root] = 1; m_td[hi] += p m_td[v]; m_td[lo] += (1-p) m_td[v]
//              (Alg. "Forward Traversal of XBDDs"); P[c False] = m_td[False terminal]
//   backward : beta(v) = P[reach False from v]: beta(True)=0, beta(False)=1,
//              beta(v) = p beta(hi) + (1-p) beta(lo) in reverse order, and
//              dP[c False]/dp_s = sum_{v: slot s} m_td(v) (beta(hi) - beta(lo))
//              (Alg. "Backward Traversal of XBDD", Lemma "backward"; the gradient of the
//              false mass, so the sign is the opposite of the paper's true-mass form)
//   scatter  : grad_a += w (-1/2) dP/dp; grad_b[j] += w dP/dp * dp/dz * q_j
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "fsmt_internal.hpp"
#include "kernels_common.hpp"

namespace fsmt {

struct CopArgs {
    const TplInfo *tpl;
    const Node *nodes;
    const BucketInfo *bucket;
    const int32_t *bucket_start;
    int32_t n_buckets;
    int32_t n_pos;
    const int32_t *pos_con;
    const int32_t *sup;
    const int32_t *atom_ptr;
    const int32_t *atom_var;
    const double *atom_coef;
    const double *atom_rhs;
    const double *atom_scale;
    const uint8_t *atom_strict;
    int32_t n_bool;
    int32_t R, R_pad, log2_rpad;   // log2_rpad valid for R_pad <= 64
    int64_t n_tasks;
    View a, b, w, unsat, ga, gb;
    float *obj;
    double kappa;
    int32_t hard;
    int32_t do_grad;
    int32_t lds_nodes, lds_slots;  // per-wave LDS geometry (max over templates)
};

// Find the bucket containing position pos (uniform across the wave).
__device__ __forceinline__ int find_bucket(const int32_t *start, int nb, int pos) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (__builtin_amdgcn_readfirstlane(start[mid]) <= pos) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <bool kGrad>
__global__ void __launch_bounds__(256) cop_kernel(CopArgs A) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int64_t wave0 = (int64_t)blockIdx.x * wpb + wib;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const int NN = A.lds_nodes + 2, SS = A.lds_slots;
    float *M = lds + (size_t)wib * (2 * NN + 4 * SS) * 64;
    float *Bm = M + NN * 64;
    float *Pp = Bm + NN * 64;
    float *Qp = Pp + SS * 64;
    float *Dp = Qp + SS * 64;
    float *Gp = Dp + SS * 64;

    for (int64_t task = wave0; task < A.n_tasks; task += n_waves) {
        int pos, r;
        if (A.R_pad <= 64) {
            const int cpw = 64 >> A.log2_rpad;
            pos = (int)(task * cpw) + (lane >> A.log2_rpad);
            r = lane & (A.R_pad - 1);
        } else {
            const int wpc = A.R_pad >> 6;
            pos = (int)(task / wpc);
            r = (int)(task % wpc) * 64 + lane;
        }
        const int pos0 = __builtin_amdgcn_readfirstlane(pos);
        const int bk = find_bucket(A.bucket_start, A.n_buckets, pos0);
        const BucketInfo B = A.bucket[bk];
        const TplInfo T = A.tpl[B.tpl];
        const int N = T.n_nodes, S = T.n_slots, NB = T.n_bslots;
        const int local = pos - B.pos_begin;
        const int c = A.pos_con[pos];
        const bool valid = (c >= 0) && (r < A.R);
        const int32_t *sup = A.sup + B.sup_base + local;

        // ---- literal probabilities (Eq. "rounding", Eq. "sampling")
        for (int s = 0; s < NB; ++s) {
            const int id = valid ? sup[(int64_t)s * B.n_pos] : 0;
            const float av = valid ? A.a.at(r, id) : 0.0f;
            Pp[s * 64 + lane] = (1.0f - av) * 0.5f;
            Qp[s * 64 + lane] = (1.0f + av) * 0.5f;
        }
        for (int s = NB; s < S; ++s) {
            float p = 0.5f, q = 0.5f, d = 0.0f;
            if (valid) {
                const int k = sup[(int64_t)s * B.n_pos] - A.n_bool;
                const double z = atom_z_exact(A.atom_ptr, A.atom_var, A.atom_coef, A.atom_rhs, k, A.b, r);
                if (A.hard) {
                    const bool t = A.atom_strict[k] ? (z < 0.0) : (z <= 0.0);
                    p = t ? 1.0f : 0.0f;
                    q = t ? 0.0f : 1.0f;
                } else {
                    const double ks = A.kappa * A.atom_scale[k];
                    const float u = (float)(z * ks);
                    const float e = 0.5f * erfcf(fabsf(u));     // the smaller of p, 1-p
                    p = (u >= 0.0f) ? e : 1.0f - e;
                    q = (u >= 0.0f) ? 1.0f - e : e;
                    if (u != u) { p = u; q = u; }              // NaN in, NaN out
                    d = -(float)(ks * 0.56418958354775628695) * expf(-u * u);   // dp/dz
                }
            }
            Pp[s * 64 + lane] = p;
            Qp[s * 64 + lane] = q;
            Dp[s * 64 + lane] = d;
        }

        // ---- forward: top-down path masses
        for (int v = 0; v < N + 2; ++v) M[v * 64 + lane] = 0.0f;
        M[T.root * 64 + lane] = 1.0f;
        const Node *nd = A.nodes + T.node_off;
        for (int v = 0; v < N; ++v) {
            const Node x = load_node(nd + v);
            const float mv = M[v * 64 + lane];
            M[x.hi * 64 + lane] += Pp[x.slot * 64 + lane] * mv;
            M[x.lo * 64 + lane] += Qp[x.slot * 64 + lane] * mv;
        }
        const float unsat = M[(N + 1) * 64 + lane];
        const float wc = valid ? A.w.at(r, c) : 0.0f;
        if (valid && A.unsat.data) A.unsat.at(r, c) = unsat;

        // objective: reduce lanes holding the same restart, then one atomic per restart
        if (A.obj) {
            float contrib = valid ? wc * unsat : 0.0f;
            if (A.R_pad < 64) {
                for (int off = 32; off >= A.R_pad; off >>= 1) contrib += __shfl_xor(contrib, off, 64);
                if (lane < A.R_pad && r < A.R) atomic_add_f32(A.obj + r, contrib);
            } else if (r < A.R) {
                atomic_add_f32(A.obj + r, contrib);
            }
        }
        if (!kGrad) continue;

        // ---- backward: bottom-up false-reaching masses and slot sensitivities
        for (int s = 0; s < S; ++s) Gp[s * 64 + lane] = 0.0f;
        Bm[N * 64 + lane] = 0.0f;
        Bm[(N + 1) * 64 + lane] = 1.0f;
        for (int v = N - 1; v >= 0; --v) {
            const Node x = load_node(nd + v);
            const float bh = Bm[x.hi * 64 + lane], bl = Bm[x.lo * 64 + lane];
            Bm[v * 64 + lane] = Pp[x.slot * 64 + lane] * bh + Qp[x.slot * 64 + lane] * bl;
            Gp[x.slot * 64 + lane] += M[v * 64 + lane] * (bh - bl);
        }
        // ---- chain rule and scatter
        if (valid) {
            for (int s = 0; s < NB; ++s) {
                const float g = wc * Gp[s * 64 + lane] * -0.5f;
                if (g != 0.0f) atomic_add_f32(&A.ga.at(r, sup[(int64_t)s * B.n_pos]), g);
            }
            for (int s = NB; s < S; ++s) {
                const float gz = wc * Gp[s * 64 + lane] * Dp[s * 64 + lane];
                if (gz == 0.0f) continue;
                const int k = sup[(int64_t)s * B.n_pos] - A.n_bool;
                for (int e = A.atom_ptr[k]; e < A.atom_ptr[k + 1]; ++e)
                    atomic_add_f32(&A.gb.at(r, A.atom_var[e]), gz * (float)A.atom_coef[e]);
            }
        }
    }
}

// ------------------------------------------------------------------ small kernels
__global__ void fill_view_kernel(View v, float value) {
    const int64_t n = (int64_t)v.rows * v.cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / v.cols), j = (int)(i % v.cols);
        v.at(r, j) = value;
    }
}

__global__ void fill_f32_kernel(float *p, int64_t n, float value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = value;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = value;
}

// One block per restart: clamp step, gradient-map norm, zero the gradient.
__global__ void __launch_bounds__(256) pgd_kernel(View a, View b, View ga, View gb, const float *lo,
                                                  const float *hi, float eta_a, float eta_b, float *gsq) {
    const int r = blockIdx.x;
    float acc = 0.0f;
    for (int i = threadIdx.x; i < a.cols; i += blockDim.x) {
        const float x = a.at(r, i);
        const float y = x - eta_a * ga.at(r, i);
        const float p = y < -1.0f ? -1.0f : (y > 1.0f ? 1.0f : y);
        a.at(r, i) = p;
        const float g = (x - p) / eta_a;
        acc += g * g;
        ga.at(r, i) = 0.0f;
    }
    for (int j = threadIdx.x; j < b.cols; j += blockDim.x) {
        const float x = b.at(r, j);
        const float y = x - eta_b * gb.at(r, j);
        const float p = y < lo[j] ? lo[j] : (y > hi[j] ? hi[j] : y);
        b.at(r, j) = p;
        const float g = (x - p) / eta_b;
        acc += g * g;
        gb.at(r, j) = 0.0f;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0 && gsq) gsq[r] = acc;
}

struct CheckArgs {
    const TplInfo *tpl;
    const Node *nodes;
    const BucketInfo *bucket;
    const int32_t *con_bucket, *con_local, *sup;
    const int32_t *atom_ptr, *atom_var;
    const double *atom_coef, *atom_rhs;
    const uint8_t *atom_strict;
    int32_t n_bool, n_cons, n_words;
    View a, b;
    uint32_t *sat_bits;
    int32_t *n_unsat;
};

// grid.x over 64-constraint groups (one wave each), grid.y over restarts.
__global__ void __launch_bounds__(256) check_kernel(CheckArgs A) {
    const int lane = threadIdx.x & 63;
    const int64_t c64 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    const int r = blockIdx.y;
    const int c = (int)c64;
    bool sat = false;
    if (c64 < A.n_cons) sat = walk_exact(A.tpl, A.nodes, A.bucket, A.con_bucket, A.con_local, A.sup, A.atom_ptr,
                                         A.atom_var, A.atom_coef, A.atom_rhs, A.atom_strict, A.n_bool, A.a, A.b,
                                         c, r);
    const uint64_t mask = __ballot(sat);
    const uint64_t valid = __ballot(c64 < A.n_cons);
    if (lane == 0 && valid) {
        const int64_t w0 = (c64 - 0) >> 5;   // c64 is a multiple of 64 on lane 0
        uint32_t *row = A.sat_bits + (int64_t)r * A.n_words;
        row[w0] = (uint32_t)mask;
        if (w0 + 1 < A.n_words) row[w0 + 1] = (uint32_t)(mask >> 32);
        atomicAdd(A.n_unsat + r, (int)__popcll(valid & ~mask));
    }
}

__global__ void verdict_kernel(View a, int8_t *x, const int32_t *n_unsat, int32_t *verdict) {
    const int r = blockIdx.x;
    if (threadIdx.x == 0) verdict[r] = n_unsat[r] == 0 ? 1 : 0;
    if (x)
        for (int i = threadIdx.x; i < a.cols; i += blockDim.x) x[(int64_t)r * a.cols + i] = a.at(r, i) < 0.0f ? -1 : 1;
}

// ------------------------------------------------------------------ host side

static fsmt_status check_view(const fsmt_view &v, int rows, int cols, const char *name, bool allow_bcast = false) {
    if (cols > 0 && rows > 0 && !v.data) return set_error(FSMT_EINVAL, "%s: null data", name);
    if (v.rows != rows || v.cols != cols)
        return set_error(FSMT_EINVAL, "%s: shape [%d][%d], expected [%d][%d]", name, v.rows, v.cols, rows, cols);
    if (v.stride_v < 0 || v.stride_r < 0) return set_error(FSMT_EINVAL, "%s: negative stride", name);
    if (cols > 1 && v.stride_v == 0) return set_error(FSMT_EINVAL, "%s: zero column stride", name);
    if (rows > 1 && v.stride_r == 0 && !allow_bcast) return set_error(FSMT_EINVAL, "%s: zero row stride", name);
    return FSMT_OK;
}

fsmt_status check_device_ptr(const void *p, int device, const char *name) {
    if (!p) return FSMT_OK;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FSMT_EINVAL, "%s: not a device pointer", name);
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return set_error(FSMT_EINVAL, "%s: not device memory", name);
    if (at.device != device) return set_error(FSMT_EINVAL, "%s: on device %d, handle on %d", name, at.device, device);
    return FSMT_OK;
}

fsmt_status select_device(const fsmt_xbdd *h) {
    if (h->host_only) return set_error(FSMT_EINVAL, "handle was compiled host-only");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return set_error(FSMT_EHIP, "hipGetDevice failed");
    if (cur != h->device) return set_error(FSMT_EINVAL, "current device %d differs from the handle's device %d", cur, h->device);
    return FSMT_OK;
}

static fsmt_status launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FSMT_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FSMT_OK;
}

static int blocks_for(int64_t n, int threads, int cap = 4096) {
    int64_t b = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

fsmt_status fill_view(const fsmt_view &v, float value, hipStream_t st) {
    if (!v.data || v.rows == 0 || v.cols == 0) return FSMT_OK;
    hipLaunchKernelGGL(fill_view_kernel, dim3(blocks_for((int64_t)v.rows * v.cols, 256)), dim3(256), 0, st,
                       View::of(v), value);
    return launch_status("fill");
}

fsmt_status fill_f32(float *p, int64_t n, float value, hipStream_t st) {
    if (!p || n <= 0) return FSMT_OK;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, value);
    return launch_status("fill");
}

static fsmt_status cop_launch(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, double kappa, fsmt_view w, float *obj,
                              fsmt_view unsat, fsmt_view ga, fsmt_view gb, bool grad, int32_t flags, hipStream_t st) {
    const int R = a.rows;
    fsmt_status rc;
    if (!h) return set_error(FSMT_EINVAL, "null handle");
    if (R <= 0) return set_error(FSMT_EINVAL, "a: no rows");
    if ((rc = check_view(a, R, h->n_bool, "a"))) return rc;
    if ((rc = check_view(b, R, h->n_real, "b"))) return rc;
    if (w.rows == 1 && R > 1 && w.stride_r == 0) {
        if ((rc = check_view(w, 1, h->n_cons, "w"))) return rc;
    } else if ((rc = check_view(w, R, h->n_cons, "w"))) {
        return rc;
    }
    if (unsat.data && (rc = check_view(unsat, R, h->n_cons, "unsat"))) return rc;
    if (grad) {
        if ((rc = check_view(ga, R, h->n_bool, "grad_a"))) return rc;
        if ((rc = check_view(gb, R, h->n_real, "grad_b"))) return rc;
    }
    if (!(kappa >= 0.0)) return set_error(FSMT_EINVAL, "kappa must be in [0, +inf]");
    if ((rc = select_device(h))) return rc;
    const void *ptrs[] = {a.data, b.data, w.data, obj, unsat.data, grad ? ga.data : nullptr, grad ? gb.data : nullptr};
    const char *names[] = {"a", "b", "w", "obj", "unsat", "grad_a", "grad_b"};
    for (int i = 0; i < 7; ++i)
        if ((rc = check_device_ptr(ptrs[i], h->device, names[i]))) return rc;

    const int NN = h->max_nodes + 2, SS = std::max(h->max_slots, 1);
    const size_t wave_bytes = (size_t)(2 * NN + 4 * SS) * 64 * sizeof(float);
    if (wave_bytes > 65536)
        return set_error(FSMT_ELIMIT, "diagram too large for the LDS-resident pass (%d nodes, %d slots)", h->max_nodes, h->max_slots);
    int wpb = (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / wave_bytes));

    if (!(flags & FSMT_ACCUMULATE)) {
        if (obj && (rc = fill_f32(obj, R, 0.0f, st))) return rc;
        if (grad && ((rc = fill_view(ga, 0.0f, st)) || (rc = fill_view(gb, 0.0f, st)))) return rc;
    }
    if (h->n_pos == 0) return FSMT_OK;

    CopArgs A{};
    A.tpl = h->d.tpl;
    A.nodes = h->d.nodes;
    A.bucket = h->d.bucket;
    A.bucket_start = h->d.bucket_start;
    A.n_buckets = h->n_buckets;
    A.n_pos = h->n_pos;
    A.pos_con = h->d.pos_con;
    A.sup = h->d.sup;
    A.atom_ptr = h->d.atom_ptr;
    A.atom_var = h->d.atom_var;
    A.atom_coef = h->d.atom_coef;
    A.atom_rhs = h->d.atom_rhs;
    A.atom_scale = h->d.atom_scale;
    A.atom_strict = h->d.atom_strict;
    A.n_bool = h->n_bool;
    A.R = R;
    if (R <= 64) {
        int rp = 1, lg = 0;
        while (rp < R) { rp <<= 1; ++lg; }
        A.R_pad = rp;
        A.log2_rpad = lg;
        A.n_tasks = (int64_t)h->n_pos * rp / 64;
    } else {
        A.R_pad = (R + 63) / 64 * 64;
        A.log2_rpad = 0;
        A.n_tasks = (int64_t)h->n_pos * (A.R_pad / 64);
    }
    A.a = View::of(a);
    A.b = View::of(b);
    A.w = View::of(w);
    A.unsat = View::of(unsat);
    A.ga = grad ? View::of(ga) : View{};
    A.gb = grad ? View::of(gb) : View{};
    A.obj = obj;
    A.kappa = kappa;
    A.hard = std::isinf(kappa) ? 1 : 0;
    A.do_grad = grad ? 1 : 0;
    A.lds_nodes = h->max_nodes;
    A.lds_slots = SS;
    const int64_t max_waves = 256 * 32;
    const int64_t waves = std::min<int64_t>(A.n_tasks, max_waves);
    const int blocks = (int)((waves + wpb - 1) / wpb);
    const size_t lds = wave_bytes * wpb;
    if (grad)
        hipLaunchKernelGGL(cop_kernel<true>, dim3(blocks), dim3(64 * wpb), lds, st, A);
    else
        hipLaunchKernelGGL(cop_kernel<false>, dim3(blocks), dim3(64 * wpb), lds, st, A);
    return launch_status("cop kernel");
}

}  // namespace fsmt

using namespace fsmt;

extern "C" {

fsmt_status cop_forward(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, double kappa, fsmt_view w, float *obj,
                        fsmt_view unsat, int32_t flags, void *stream) {
    clear_error();
    if (!obj) return set_error(FSMT_EINVAL, "obj is required");
    return cop_launch(h, a, b, kappa, w, obj, unsat, fsmt_view{}, fsmt_view{}, false, flags, (hipStream_t)stream);
}

fsmt_status cop_backward(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, double kappa, fsmt_view w, float *obj,
                         fsmt_view grad_a, fsmt_view grad_b, int32_t flags, void *stream) {
    clear_error();
    return cop_launch(h, a, b, kappa, w, obj, fsmt_view{}, grad_a, grad_b, true, flags, (hipStream_t)stream);
}

fsmt_status pgd_step(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, fsmt_view grad_a, fsmt_view grad_b, float eta_a,
                     float eta_b, float *gmap_sq, int32_t flags, void *stream) {
    clear_error();
    (void)flags;
    if (!h) return set_error(FSMT_EINVAL, "null handle");
    const int R = a.rows;
    fsmt_status rc;
    if (R <= 0) return set_error(FSMT_EINVAL, "a: no rows");
    if ((rc = check_view(a, R, h->n_bool, "a")) || (rc = check_view(b, R, h->n_real, "b")) ||
        (rc = check_view(grad_a, R, h->n_bool, "grad_a")) || (rc = check_view(grad_b, R, h->n_real, "grad_b")))
        return rc;
    if (!(eta_a > 0.0f) || !(eta_b > 0.0f)) return set_error(FSMT_EINVAL, "step sizes must be positive");
    if ((rc = select_device(h))) return rc;
    const void *ptrs[] = {a.data, b.data, grad_a.data, grad_b.data, gmap_sq};
    const char *names[] = {"a", "b", "grad_a", "grad_b", "gmap_sq"};
    for (int i = 0; i < 5; ++i)
        if ((rc = check_device_ptr(ptrs[i], h->device, names[i]))) return rc;
    hipLaunchKernelGGL(pgd_kernel, dim3(R), dim3(256), 0, (hipStream_t)stream, View::of(a), View::of(b),
                       View::of(grad_a), View::of(grad_b), h->d.real_lo, h->d.real_hi, eta_a, eta_b, gmap_sq);
    return launch_status("pgd kernel");
}

fsmt_status round_and_check(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, int8_t *x, uint32_t *sat_bits,
                            int32_t *n_unsat, int32_t *verdict, void *stream) {
    clear_error();
    if (!h) return set_error(FSMT_EINVAL, "null handle");
    const int R = a.rows;
    fsmt_status rc;
    if (R <= 0) return set_error(FSMT_EINVAL, "a: no rows");
    if ((rc = check_view(a, R, h->n_bool, "a")) || (rc = check_view(b, R, h->n_real, "b"))) return rc;
    if (!sat_bits || !n_unsat || !verdict) return set_error(FSMT_EINVAL, "sat_bits, n_unsat and verdict are required");
    if (R > 65535) return set_error(FSMT_ELIMIT, "at most 65535 rows");
    if ((rc = select_device(h))) return rc;
    const void *ptrs[] = {a.data, b.data, x, sat_bits, n_unsat, verdict};
    const char *names[] = {"a", "b", "x", "sat_bits", "n_unsat", "verdict"};
    for (int i = 0; i < 6; ++i)
        if ((rc = check_device_ptr(ptrs[i], h->device, names[i]))) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(R, 256)), dim3(256), 0, st, n_unsat, (int64_t)R, 0);
    if ((rc = launch_status("fill"))) return rc;
    CheckArgs A{};
    A.tpl = h->d.tpl;
    A.nodes = h->d.nodes;
    A.bucket = h->d.bucket;
    A.con_bucket = h->d.con_bucket;
    A.con_local = h->d.con_local;
    A.sup = h->d.sup;
    A.atom_ptr = h->d.atom_ptr;
    A.atom_var = h->d.atom_var;
    A.atom_coef = h->d.atom_coef;
    A.atom_rhs = h->d.atom_rhs;
    A.atom_strict = h->d.atom_strict;
    A.n_bool = h->n_bool;
    A.n_cons = h->n_cons;
    A.n_words = (h->n_cons + 31) / 32;
    A.a = View::of(a);
    A.b = View::of(b);
    A.sat_bits = sat_bits;
    A.n_unsat = n_unsat;
    if (h->n_cons > 0) {
        const int gx = (int)((h->n_cons + 255) / 256);
        hipLaunchKernelGGL(check_kernel, dim3(gx, R), dim3(256), 0, st, A);
        if ((rc = launch_status("check kernel"))) return rc;
    }
    hipLaunchKernelGGL(verdict_kernel, dim3(R), dim3(256), 0, st, View::of(a), x, n_unsat, verdict);
    return launch_status("verdict kernel");
}

}  // extern "C"
