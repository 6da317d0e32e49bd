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

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "fsmt_internal.hpp"
#include "eval_task.hpp"

namespace fsmt {

struct CopArgs {
    TabView T;
    int32_t R, R_pad, log2_rpad;   // log2_rpad valid for R_pad <= 64
    int64_t n_tasks;
    View a, b, w, unsat, ga, gb;
    float *obj;
    double kappa;
    int32_t hard;
    int32_t lds_nodes, lds_slots;  // per-wave LDS geometry (max over templates)
};

template <bool kGrad, int V, int kCF>
__global__ void __launch_bounds__(256) cop_kernel(CopArgs A) {
    using Ms = typename MsgOf<V>::type;
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63;
    const int wib = wave_id();
    const int wpb = blockDim.x >> 6;
    const int64_t wave0 = (int64_t)blockIdx.x * wpb + wib;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    const int NN = A.lds_nodes + 2, SS = A.lds_slots;
    FSMT_MSG_STORE(Ms, W, lds + (size_t)wib * (2 * NN + 4 * SS) * 64, NN, SS, lane);
    const GlobalState st{A.a, A.b};
    const GlobalScatter sc{A.ga, A.gb, A.R_pad < 64 ? A.R_pad : 64};
    float oacc = 0.0f;   // objective partial of this lane's restart (R_pad <= 64: fixed per lane)

    for (int64_t task = wave0; task < A.n_tasks; task += n_waves) {
        int pos, r;
        if (A.R_pad <= 64) {
            pos = (int)(task * (64 >> A.log2_rpad)) + (lane >> A.log2_rpad);
            r = lane & (A.R_pad - 1);
        } else {
            const int wpc = A.R_pad >> 6;
            pos = (int)(task / wpc);
            r = (int)(task % wpc) * 64 + lane;
        }
        const TaskCtx t = task_ctx(A.T, pos, r, r < A.R);
        if (t.B.big) continue;   // evaluated by cop_level_kernel
        const float wc = t.valid ? A.w.at(r, t.c) : 0.0f;   // requested before the forward pass
        const float unsat = task_eval<kGrad, kCF, true>(A.T, t, st, A.kappa, A.hard != 0, wc, sc, W, lane);
        if (t.valid && A.unsat.data) A.unsat.at(r, t.c) = unsat;
        if (A.obj) {
            if (A.R_pad <= 64) {
                oacc += wc * unsat;
            } else if (r < A.R) {
                atomic_add_f32(A.obj + r, wc * unsat);
            }
        }
    }
    // objective: reduce lanes holding the same restart, one atomic per restart and wave
    if (A.obj && A.R_pad <= 64) {
        for (int off = 32; off >= A.R_pad; off >>= 1) oacc += __shfl_xor(oacc, off, 64);
        if (lane < A.R_pad && lane < A.R && oacc != 0.0f) atomic_add_f32(A.obj + lane, oacc);
    }
}

// Restarts in groups of G (1, 2 or 4; small diagrams, register message store): each
// workgroup serves one group, its waves holding 64 / G constraints x G restarts, and adds the
// gradient into an LDS copy of the group's n + m variables x G restarts (restart-minor),
// written out once as the workgroup's partial row; sum_rows_kernel adds the rows of each
// group. The group's point is copied into LDS too, so the state gathers are LDS reads. This
// replaces the device-scope atomics on the caller's gradient, which are performed at the
// memory side (one line write per variable and wave-wide atomic).
struct LdsStateG {
    const float *a, *b;
    int G, r0;
    __device__ __forceinline__ float av(int r, int i) const { return a[i * G + ((r - r0) & (G - 1))]; }
    __device__ __forceinline__ float bv(int r, int j) const { return b[j * G + ((r - r0) & (G - 1))]; }
};
struct LdsScatterG {
    float *ga, *gb;
    int G, r0;
    __device__ __forceinline__ void add_a(int r, int i, float g, int) const {
        if (i >= 0 && g != 0.0f) atomicAdd(ga + i * G + ((r - r0) & (G - 1)), g);
    }
    __device__ __forceinline__ void add_b(int r, int j, float g, int) const {
        if (j >= 0 && g != 0.0f) atomicAdd(gb + j * G + ((r - r0) & (G - 1)), g);
    }
    __device__ __forceinline__ void add_b_direct(int r, int j, float g) const {
        atomicAdd(gb + j * G + ((r - r0) & (G - 1)), g);
    }
};

template <int kCF, int G>
__global__ void __launch_bounds__(1024) cop_lds_grad_kernel(CopArgs A, float *part, int n_groups) {
    using Ms = typename MsgOf<kMsgSmall>::type;
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63;
    const int wib = wave_id();
    const int wpb = blockDim.x >> 6;
    const int n = A.T.n_bool, nm = A.T.n_bool + A.T.n_real;
    // workgroup w of every group takes the same tasks; blocks are dealt to the XCDs round
    // robin, so with group-major numbering and a multiple of 8 workgroups per group those
    // workgroups share an XCD and its L2 serves the tables to all groups
    const int64_t n_wg = gridDim.x / n_groups, wg = blockIdx.x % n_wg;
    const int group = (int)(blockIdx.x / n_wg), r0 = group * G;
    float *const sy = lds + nm * G;   // a then b, [variable][G]
    // the point: four elements per thread requested together, then stored
    for (int e0 = threadIdx.x; e0 < nm * G; e0 += 4 * blockDim.x) {
        float x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * (int)blockDim.x, v = e / G, r = r0 + (e - v * G);
            x[q] = (e < nm * G && r < A.R) ? (v < n ? (float)A.a.at(r, v) : (float)A.b.at(r, v - n)) : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * (int)blockDim.x;
            if (e < nm * G) {
                lds[e] = 0.0f;
                sy[e] = x[q];
            }
        }
    }
    __syncthreads();
    FSMT_MSG_STORE(Ms, W, nullptr, 0, 0, lane);
    const LdsStateG st{sy, sy + n * G, G, r0};
    const LdsScatterG sc{lds, lds + n * G, G, r0};
    const int64_t n_tasks = (int64_t)A.T.n_pos * G / 64;
    const int r = r0 + (lane & (G - 1));
    float oacc = 0.0f;
    for (int64_t task = wg * wpb + wib; task < n_tasks; task += n_wg * wpb) {
        const TaskCtx t = task_ctx(A.T, (int)(task * (64 / G)) + lane / G, r, r < A.R);
        if (t.B.big) continue;   // evaluated by cop_level_kernel
        const float wc = t.valid ? A.w.at(r, t.c) : 0.0f;   // requested before the forward pass
        const float unsat = task_eval<true, kCF, true>(A.T, t, st, A.kappa, A.hard != 0, wc, sc, W, lane);
        if (t.valid && A.unsat.data) A.unsat.at(r, t.c) = unsat;
        oacc += wc * unsat;
    }
    if (A.obj) {   // lanes G apart hold the same restart
        for (int off = 32; off >= G; off >>= 1) oacc += __shfl_xor(oacc, off, 64);
        if (lane < G && r0 + lane < A.R && oacc != 0.0f) atomic_add_f32(A.obj + r0 + lane, oacc);
    }
    __syncthreads();
    float *row = part + (int64_t)blockIdx.x * nm * G;
    for (int e = threadIdx.x; e < nm * G; e += blockDim.x) row[e] = lds[e];
}

// The groups' gradients from the workgroups' partial rows (row b belongs to group
// b / n_wg): 64 elements per block, the rows split over 16 stripes and the stripes'
// sums added in LDS; stored into (or added to) the caller's views.
__global__ void __launch_bounds__(1024) sum_rows_kernel(const float *part, int n_groups, int n_wg, int G, int R, int n,
                                                        int m, View ga, View gb, int accumulate) {
    __shared__ float red[16][64];
    const int c = threadIdx.x & 63, s = threadIdx.x >> 6;
    const int nm = n + m, group = blockIdx.y;
    const int e = blockIdx.x * 64 + c;
    float acc = 0.0f;
    if (e < nm * G) {
        // a stripe's first 16 rows are requested together (one round trip, not 16)
        const float *col = part + (int64_t)group * n_wg * nm * G + e;
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int w = s + 16 * q;
            v[q] = w < n_wg ? col[(int64_t)w * nm * G] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) acc += v[q];
        for (int w = s + 256; w < n_wg; w += 16) acc += col[(int64_t)w * nm * G];
    }
    red[s][c] = acc;
    __syncthreads();
    const int v = e / G, r = group * G + (e - v * G);
    if (s == 0 && e < nm * G && r < R) {
        float t = 0.0f;
        for (int q = 0; q < 16; ++q) t += red[q][c];
        gref<float> dst = v < n ? ga.at(r, v) : gb.at(r, v - n);
        if (accumulate) dst += t; else dst = t;
    }
}

// ------------------------------------------------------------------ big diagrams
// Level-synchronous passes (see level_eval): one wavefront per (big constraint, chunk of
// restarts); the wave stages the constraint's node table in its LDS rows once and evaluates
// the chunk's restarts one after the other, keeping the objective's partial sums in lanes.
struct LevelArgs {
    TabView T;
    cptr<int32_t> lev, big_pos;
    int32_t n_big, R, chunk;
    View a, b, w, unsat, ga, gb;
    float *obj;
    double kappa;
    int32_t hard;
    int32_t lds_nodes, lds_slots;   // per-wave LDS rows (max over big templates)
};

template <bool kGrad>
__global__ void __launch_bounds__(256) cop_level_kernel(LevelArgs A) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63;
    const int wib = wave_id();
    const int wpb = blockDim.x >> 6;
    const LevelRows W = LevelRows::at(lds + (size_t)wib * level_wave_floats(A.lds_nodes, A.lds_slots), A.lds_nodes,
                                      A.lds_slots);
    const GlobalState st{A.a, A.b};
    const GlobalScatter sc{A.ga, A.gb, 64};
    const int chunks = (A.R + A.chunk - 1) / A.chunk;
    const int64_t n_tasks = (int64_t)A.n_big * chunks;
    WaveObjAcc oa{A.obj};
    // chunk-major task order: a wave's consecutive tasks share their restart chunk
    for (int64_t task = (int64_t)blockIdx.x * wpb + wib; task < n_tasks; task += (int64_t)gridDim.x * wpb) {
        const int ci = (int)(task / A.n_big), q = (int)(task - (int64_t)ci * A.n_big);
        const int r0 = ci * A.chunk, r1 = r0 + A.chunk < A.R ? r0 + A.chunk : A.R;
        oa.begin(r0, r1 - r0, lane);
        const LevelCtx L = level_ctx(A.T, A.lev, A.big_pos[q]);
        level_stage_nodes(A.T, L, W, lane);
        for (int r = r0; r < r1; ++r) {
            const float wc = A.w.at(r, L.c);
            const float unsat = level_eval(A.T, L, st, sc, r, A.kappa, A.hard != 0, wc, kGrad, W, lane);
            if (lane == 0 && A.unsat.data) A.unsat.at(r, L.c) = unsat;
            oa.add(r - r0, wc * unsat, lane);
        }
    }
    oa.flush(lane);
}

// ------------------------------------------------------------------ small kernels
// out(r, v) (+)= stage[v * R + r]: the gradient accumulated restart-contiguous (see
// cop_launch) moved into the caller's view.
__global__ void unstage_kernel(View out, const float *stage, int R, int cols, int accumulate) {
    const int64_t n = (int64_t)R * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int v = (int)(e / R), r = (int)(e - (int64_t)v * R);
        const float g = stage[e];
        if (accumulate) out.at(r, v) += g; else out.at(r, v) = g;
    }
}

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

// One block per restart: clamp / project step, gradient-map norm, zero the gradient.
__global__ void __launch_bounds__(256) pgd_kernel(View a, View b, View ga, View gb, cptr<float> lo,
                                                  cptr<float> hi, float eta_a, float eta_b, float *gsq,
                                                  HalfSpaces hs) {
    extern __shared__ float sm[];
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
    if (hs.n == 0) {
        for (int j = threadIdx.x; j < b.cols; j += blockDim.x) {
            const float x = b.at(r, j);
            const float y = x - eta_b * gb.at(r, j);
            const float p = y < lo[j] ? lo[j] : (y > hi[j] ? hi[j] : y);
            b.at(r, j) = p;
            const float g = (x - p) / eta_b;
            acc += g * g;
            gb.at(r, j) = 0.0f;
        }
    } else {
        const int m = b.cols;
        float *y = sm, *pb = sm + m, *ph = sm + 2 * m;
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            y[j] = b.at(r, j) - eta_b * gb.at(r, j);
            gb.at(r, j) = 0.0f;
        }
        project_dykstra(y, pb, ph, lo, hi, m, hs);
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            const float x = b.at(r, j), p = y[j];
            b.at(r, j) = p;
            const float g = (x - p) / eta_b;
            acc += g * g;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0 && gsq) gsq[r] = acc;
}

struct CheckArgs {
    TabView T;
    int32_t n_words;
    View a, b;
    uint32_t *sat_bits;
    int32_t *n_unsat;
};

// grid.x over 64-constraint groups (one wave each), grid.y over restarts.
__global__ void __launch_bounds__(256) check_kernel(CheckArgs A) {
    const int lane = threadIdx.x & 63;
    const int64_t c64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const GlobalState st{A.a, A.b};
    bool sat = false;
    if (c64 < A.T.n_cons) sat = walk_state(A.T, st, (int)c64, r);
    const uint64_t mask = __ballot(sat);
    const uint64_t valid = __ballot(c64 < A.T.n_cons);
    if (lane == 0 && valid) {
        const int64_t w0 = c64 >> 5;   // lane 0 holds a multiple of 64
        uint32_t *row = A.sat_bits + (int64_t)r * A.n_words;
        row[w0] = (uint32_t)mask;
        if (w0 + 1 < A.n_words) row[w0 + 1] = (uint32_t)(mask >> 32);
        atomicAdd(A.n_unsat + r, (int)__popcll(valid & ~mask));
    }
}

// ERWA update of Alg. "CLS with Annealing" for level t (1-based), one block per restart.
__global__ void __launch_bounds__(1024) erwa_kernel(int C, const uint32_t *bits, float *w, float *hist, int t, float rho,
                                                    float gamma, int tau, int normalize) {
    const int r = blockIdx.x, nw = (C + 31) >> 5;
    const bool update = (t % tau) == 0;
    float *wr = w + (int64_t)r * C, *hr = hist + (int64_t)r * C;
    const uint32_t *br = bits + (int64_t)r * nw;
    float ws = 0.0f;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const float viol = ((br[c >> 5] >> (c & 31)) & 1u) ? 0.0f : 1.0f;
        float h = rho * hr[c] + viol, wv = wr[c];
        if (update) {
            wv *= powf(gamma, h);
            h = 1.0f;
            wr[c] = wv;
        }
        hr[c] = h;
        ws += wv;
    }
    ws = block_sum(ws);
    if (update && normalize) {
        const float scale = (float)C / ws;
        for (int c = threadIdx.x; c < C; c += blockDim.x) wr[c] *= scale;
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

HalfSpaces halfspaces_of(const fsmt_xbdd *h) {
    return HalfSpaces{as_cptr(h->d.hs_ptr), as_cptr(h->d.hs_var), as_cptr(h->d.hs_coef), as_cptr(h->d.hs_rhs),
                      as_cptr(h->d.hs_inv), as_cptr(h->d.hs_cstart), h->n_hs, h->hs_nnz, h->n_hs_colors,
                      h->hs_separable};
}

static fsmt_status launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FSMT_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FSMT_OK;
}

template <bool kGrad, int kCF>
static void launch_cop_v(int msg, dim3 g, dim3 bl, size_t lds, hipStream_t st, const CopArgs &A) {
    if (msg == kMsgSmall) hipLaunchKernelGGL((cop_kernel<kGrad, kMsgSmall, kCF>), g, bl, 0, st, A);
    else if (msg == kMsgMedium) hipLaunchKernelGGL((cop_kernel<kGrad, kMsgMedium, kCF>), g, bl, 0, st, A);
    else if (msg == kMsgLarge) hipLaunchKernelGGL((cop_kernel<kGrad, kMsgLarge, kCF>), g, bl, 0, st, A);
    else hipLaunchKernelGGL((cop_kernel<kGrad, kMsgLds, kCF>), g, bl, lds, st, A);
}
template <bool kGrad>
static void launch_cop(int cf, int msg, dim3 g, dim3 bl, size_t lds, hipStream_t st, const CopArgs &A) {
    if (cf == 0) launch_cop_v<kGrad, 0>(msg, g, bl, lds, st, A);
    else if (cf == 1) launch_cop_v<kGrad, 1>(msg, g, bl, lds, st, A);
    else if (cf == 2) launch_cop_v<kGrad, 2>(msg, g, bl, lds, st, A);
    else launch_cop_v<kGrad, 3>(msg, g, bl, lds, st, A);
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

fsmt_status fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t st) {
    if (!p || n <= 0) return FSMT_OK;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, value);
    return launch_status("fill");
}

fsmt_status fill_f32(float *p, int64_t n, float value, hipStream_t st) {
    if (!p || n <= 0) return FSMT_OK;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, value);
    return launch_status("fill");
}

// Dynamic LDS the gradient-in-LDS kernels may take: the device's per-block maximum, opted
// into once for every instantiation (64 KB if the device reports no more).
static size_t lds_grad_budget() {
    static size_t budget = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, v = 0;
        size_t b = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && (size_t)v > b)
            b = (size_t)v;
        const void *fns[] = {(const void *)cop_lds_grad_kernel<0, 1>, (const void *)cop_lds_grad_kernel<1, 1>,
                             (const void *)cop_lds_grad_kernel<2, 1>, (const void *)cop_lds_grad_kernel<0, 2>,
                             (const void *)cop_lds_grad_kernel<1, 2>, (const void *)cop_lds_grad_kernel<2, 2>,
                             (const void *)cop_lds_grad_kernel<0, 4>, (const void *)cop_lds_grad_kernel<1, 4>,
                             (const void *)cop_lds_grad_kernel<2, 4>};
        for (const void *f : fns)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b) != hipSuccess) {
                (void)hipGetLastError();
                b = 65536;
            }
        budget = b;
    });
    return budget;
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

    // one lane per constraint for the small diagrams, one wavefront per (constraint,
    // restart) for the big ones
    const int NN = h->small_max_nodes + 2, SS = std::max(h->small_max_slots, 1);
    const int msg = msg_variant(h->small_max_nodes, h->small_max_slots, lds_store(h), h->all_inline);
    const size_t wave_bytes = msg == kMsgLds ? WaveScratch::bytes(NN, SS) : 0;
    const int wpb = wave_bytes ? (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / wave_bytes)) : 4;
    const size_t level_wave_bytes = level_wave_floats(h->big_max_nodes, std::max(h->big_max_slots, 1)) * sizeof(float);
    if (h->n_big > 0 && level_wave_bytes > 65536)
        return set_error(FSMT_ELIMIT, "diagram too large for the level-synchronous pass (%d nodes, %d slots)",
                         h->big_max_nodes, h->big_max_slots);

    // With several restarts in a wavefront's lanes, the lanes of one constraint add into the
    // same variable of consecutive restarts. Device-scope float atomics are performed past
    // the per-XCD L2, one memory transaction per cache line touched, so when the caller's
    // gradient rows are not restart-contiguous the sums go to a restart-contiguous stage
    // ([n + m][R], one line per variable and 16 restarts) and are moved into the caller's
    // views afterwards. With up to 16 restarts over small diagrams with a register message
    // store, the gradient is summed per workgroup in LDS for groups of up to 4 restarts
    // (cop_lds_grad_kernel) and the workgroups' rows are added afterwards, one row per CU;
    // where it applies it replaces the stage. Both are taken only for instances of at
    // least 8 tasks (64-position groups) per CU: on smaller ones the atomics cost little and
    // the extra allocation and launches would dominate the call.
    const int n = h->n_bool, m = h->n_real;
    int n_cu = 256;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    const bool large = (int64_t)h->n_pos / 64 >= (int64_t)8 * n_cu;
    bool stage = grad && large && R >= 4 && R <= 64 && (int64_t)(n + m) * R > 0 &&
                 !(ga.stride_r == 1 && gb.stride_r == 1);
    const int cf = closed_level(h);
    // restarts per LDS group: the largest of 4, 2, 1 not above R's padding whose gradient and
    // point copies (8 (n + m) G bytes) fit the workgroup's LDS
    const size_t lds_cap = lds_grad_budget();
    int gsz = 4;
    while (gsz > 1 && (gsz / 2 >= R || (size_t)8 * (n + m) * gsz > lds_cap)) gsz /= 2;
    const bool lds_grad = grad && large && R <= 16 && msg == kMsgSmall && cf <= 2 && h->n_big < h->n_cons &&
                          n + m > 0 && (size_t)8 * (n + m) * gsz <= lds_cap;
    if (lds_grad) stage = false;
    const int n_groups = lds_grad ? (R + gsz - 1) / gsz : 0;
    // workgroups per group: a multiple of 8 (the XCDs) where the CUs allow
    const int grad_wg = lds_grad ? (n_cu / n_groups >= 8 ? n_cu / n_groups / 8 * 8 : std::max(1, n_cu / n_groups)) : 0;
    const int grad_rows = n_groups * grad_wg;
    struct Stage {   // freed stream-ordered after whatever the call enqueued
        float *p = nullptr;
        hipStream_t st = nullptr;
        ~Stage() {
            if (p) (void)hipFreeAsync(p, st);
        }
    } sg;
    sg.st = st;
    if (lds_grad) {
        if (hipMallocAsync((void **)&sg.p, sizeof(float) * (size_t)(n + m) * gsz * grad_rows, st) != hipSuccess) {
            (void)hipGetLastError();
            sg.p = nullptr;
            return set_error(FSMT_ENOMEM, "gradient rows allocation failed");
        }
    }
    if (stage) {
        if (hipMallocAsync((void **)&sg.p, sizeof(float) * (size_t)(n + m) * R, st) != hipSuccess) {
            (void)hipGetLastError();
            sg.p = nullptr;
            return set_error(FSMT_ENOMEM, "gradient stage allocation failed");
        }
        if ((rc = fill_f32(sg.p, (int64_t)(n + m) * R, 0.0f, st))) return rc;
    }
    float *const sbuf = sg.p;
    if (!(flags & FSMT_ACCUMULATE)) {
        if (obj && (rc = fill_f32(obj, R, 0.0f, st))) return rc;
        if (grad && !stage && !lds_grad && ((rc = fill_view(ga, 0.0f, st)) || (rc = fill_view(gb, 0.0f, st))))
            return rc;
    }
    if (h->n_pos == 0) {
        if (stage) {
            hipLaunchKernelGGL(unstage_kernel, dim3(blocks_for((int64_t)R * n, 256)), dim3(256), 0, st, View::of(ga),
                               (const float *)sbuf, R, n, flags & FSMT_ACCUMULATE);
            hipLaunchKernelGGL(unstage_kernel, dim3(blocks_for((int64_t)R * m, 256)), dim3(256), 0, st, View::of(gb),
                               (const float *)(sbuf + (size_t)n * R), R, m, flags & FSMT_ACCUMULATE);
        }
        return launch_status("gradient unstage");
    }

    CopArgs A{};
    A.T = TabView::of(h);
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
    if (stage) {
        A.ga = View{as_gptr(sbuf), R, n, 1, R};
        A.gb = View{as_gptr(sbuf + (size_t)n * R), R, m, 1, R};
    }
    A.obj = obj;
    A.kappa = kappa;
    A.hard = std::isinf(kappa) ? 1 : 0;
    A.lds_nodes = h->small_max_nodes;
    A.lds_slots = SS;
    const int64_t max_waves = 256 * 32;
    const int64_t waves = std::min<int64_t>(A.n_tasks, max_waves);
    const int blocks = (int)((waves + wpb - 1) / wpb);
    const size_t lds = wave_bytes * wpb;
    const dim3 g(blocks), bl(64 * wpb);
    if (lds_grad) {
        const size_t glds = (size_t)8 * (n + m) * gsz;   // gradient and point, [variable][G] each
        const dim3 gg(grad_rows), gb1(1024);
        if (gsz == 1) {
            if (cf == 0) hipLaunchKernelGGL((cop_lds_grad_kernel<0, 1>), gg, gb1, glds, st, A, sbuf, n_groups);
            else if (cf == 1) hipLaunchKernelGGL((cop_lds_grad_kernel<1, 1>), gg, gb1, glds, st, A, sbuf, n_groups);
            else hipLaunchKernelGGL((cop_lds_grad_kernel<2, 1>), gg, gb1, glds, st, A, sbuf, n_groups);
        } else if (gsz == 2) {
            if (cf == 0) hipLaunchKernelGGL((cop_lds_grad_kernel<0, 2>), gg, gb1, glds, st, A, sbuf, n_groups);
            else if (cf == 1) hipLaunchKernelGGL((cop_lds_grad_kernel<1, 2>), gg, gb1, glds, st, A, sbuf, n_groups);
            else hipLaunchKernelGGL((cop_lds_grad_kernel<2, 2>), gg, gb1, glds, st, A, sbuf, n_groups);
        } else {
            if (cf == 0) hipLaunchKernelGGL((cop_lds_grad_kernel<0, 4>), gg, gb1, glds, st, A, sbuf, n_groups);
            else if (cf == 1) hipLaunchKernelGGL((cop_lds_grad_kernel<1, 4>), gg, gb1, glds, st, A, sbuf, n_groups);
            else hipLaunchKernelGGL((cop_lds_grad_kernel<2, 4>), gg, gb1, glds, st, A, sbuf, n_groups);
        }
        if ((rc = launch_status("cop kernel (gradient in LDS)"))) return rc;
        hipLaunchKernelGGL(sum_rows_kernel, dim3(((n + m) * gsz + 63) / 64, n_groups), dim3(1024), 0, st,
                           (const float *)sbuf, n_groups, grad_wg, gsz, R, n, m, View::of(ga), View::of(gb),
                           flags & FSMT_ACCUMULATE);
        if ((rc = launch_status("gradient rows"))) return rc;
    } else if (h->n_big < h->n_cons) {
        if (grad)
            launch_cop<true>(cf, msg, g, bl, lds, st, A);
        else
            launch_cop<false>(cf, msg, g, bl, lds, st, A);
        if ((rc = launch_status("cop kernel"))) return rc;
    }
    if (h->n_big > 0) {
        LevelArgs L{};
        L.T = A.T;
        L.lev = as_cptr(h->d.lev);
        L.big_pos = as_cptr(h->d.big_pos);
        L.n_big = h->n_big;
        L.R = R;
        L.a = A.a;
        L.b = A.b;
        L.w = A.w;
        L.unsat = A.unsat;
        L.ga = A.ga;
        L.gb = A.gb;
        L.obj = obj;
        L.kappa = kappa;
        L.hard = A.hard;
        L.lds_nodes = h->big_max_nodes;
        L.lds_slots = std::max(h->big_max_slots, 1);
        L.chunk = level_chunk((int64_t)h->n_big * R, n_cu);
        const int lwpb = (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / level_wave_bytes));
        const int64_t ltasks = (int64_t)h->n_big * ((R + L.chunk - 1) / L.chunk);
        const int lblocks = (int)std::min<int64_t>((ltasks + lwpb - 1) / lwpb, (int64_t)256 * 16);
        if (grad)
            hipLaunchKernelGGL(cop_level_kernel<true>, dim3(lblocks), dim3(64 * lwpb), level_wave_bytes * lwpb, st, L);
        else
            hipLaunchKernelGGL(cop_level_kernel<false>, dim3(lblocks), dim3(64 * lwpb), level_wave_bytes * lwpb, st, L);
        if ((rc = launch_status("cop level kernel"))) return rc;
    }
    if (stage) {
        hipLaunchKernelGGL(unstage_kernel, dim3(blocks_for((int64_t)R * n, 256)), dim3(256), 0, st, View::of(ga),
                           (const float *)sbuf, R, n, flags & FSMT_ACCUMULATE);
        hipLaunchKernelGGL(unstage_kernel, dim3(blocks_for((int64_t)R * m, 256)), dim3(256), 0, st, View::of(gb),
                           (const float *)(sbuf + (size_t)n * R), R, m, flags & FSMT_ACCUMULATE);
        if ((rc = launch_status("gradient unstage"))) return rc;
    }
    return FSMT_OK;
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
    const HalfSpaces hs = halfspaces_of(h);
    const size_t lds = hs.n ? (size_t)(2 * h->n_real + hs.nnz) * sizeof(float) : 0;
    if (lds > 65536) return set_error(FSMT_ELIMIT, "projection onto %d half-spaces over %d reals exceeds LDS", hs.n, h->n_real);
    hipLaunchKernelGGL(pgd_kernel, dim3(R), dim3(256), lds, (hipStream_t)stream, View::of(a), View::of(b),
                       View::of(grad_a), View::of(grad_b), as_cptr(h->d.real_lo), as_cptr(h->d.real_hi), eta_a, eta_b,
                       gmap_sq, hs);
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
    A.T = TabView::of(h);
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

fsmt_status erwa_update(const fsmt_xbdd *h, int32_t R, const uint32_t *sat_bits, float *w, float *hist, int32_t level,
                        float rho, float gamma, int32_t tau, int32_t normalize, void *stream) {
    clear_error();
    if (!h) return set_error(FSMT_EINVAL, "null handle");
    if (R <= 0 || R > 65535) return set_error(FSMT_EINVAL, "R must be in [1, 65535]");
    if (!sat_bits || !w || !hist) return set_error(FSMT_EINVAL, "null pointer");
    if (tau < 1 || level < 1 || !(gamma > 0.0f) || !(rho >= 0.0f)) return set_error(FSMT_EINVAL, "bad ERWA parameters");
    fsmt_status rc;
    if ((rc = select_device(h))) return rc;
    const void *ptrs[] = {sat_bits, w, hist};
    const char *names[] = {"sat_bits", "w", "hist"};
    for (int i = 0; i < 3; ++i)
        if ((rc = check_device_ptr(ptrs[i], h->device, names[i]))) return rc;
    if (h->n_cons == 0) return FSMT_OK;
    hipLaunchKernelGGL(erwa_kernel, dim3(R), dim3(1024), 0, (hipStream_t)stream, h->n_cons, sat_bits, w, hist, level, rho,
                       gamma, tau, normalize);
    return launch_status("erwa kernel");
}

}  // extern "C"
