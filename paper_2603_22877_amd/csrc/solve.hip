// Batched annealed solver (Alg. "CLS with Annealing" around the PGD loop of Alg.
// "FourierSMT"), fused on the device.
//
// Persistent schedule: one workgroup per (instance, restart). The restart's relaxed state
// (a, b), its gradient and the projection work arrays stay in LDS for the whole launch, so
// the gradient scatter uses LDS atomics and no global atomic is issued. Per PGD step the
// workgroup's waves sweep the instance's constraint buckets (lane = constraint, uniform
// diagram shape per wave), then project (clamp a; box + unit atoms for b), and reduce the
// gradient map norm. At the end of each level the workgroup rounds, checks every
// constraint exactly, updates the ERWA history and weights of its restart (plain loads and
// stores: the workgroup owns the row), and stops once no constraint is violated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "eval_task.hpp"
#include "solve_grid.hpp"

namespace fsmt {

constexpr int kMaxLevels = 128;

struct InstDesc {
    TabView T;
    HalfSpaces hs;
    gptr<float> a, b;
    int64_t a_sr, b_sr;
    gptr<float> w, hist;
    gptr<uint32_t> sat_bits;
    gptr<int32_t> n_unsat, verdict, level_done, steps_done;
    gptr<float> obj;
    gptr<float> part;       // [R][2][k][n + m + 1] partial gradients and objective (k > 1)
    gptr<int32_t> bar;      // [R] cluster barrier counters (k > 1)
    gptr<int32_t> ctl;      // [R][2][2] level result published by rank 0: n_unsat, stop (k > 1)
    int32_t R, wg_base, k, pad;
};

struct SolveParams {
    int32_t n_inst, n_levels, steps, tau;
    int32_t normalize, stop_mode, lds_nodes, lds_slots;
    float eta_a, eta_b, eps2, rho, gamma;
    int32_t state_floats;   // LDS floats reserved for state (max over instances)
    int32_t waves;
    int32_t pad;
    double kappas[kMaxLevels];
};

__device__ __forceinline__ int find_inst(const InstDesc *I, int n, int wg) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (__builtin_amdgcn_readfirstlane(I[mid].wg_base) <= wg) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Exchange between the k workgroups that share one restart. Partial gradients, level
// results and the barrier counter all use agent-scope atomic accesses, which are performed
// at the device's coherence point (past the per-XCD L2 caches). So no L2 write-back or
// invalidate is needed: a workgroup makes its stores complete (s_waitcnt) before it
// arrives, and reads the others' values only after it has seen every arrival. The
// compiler keeps the accesses in program order around the barrier (signal fences).
__device__ __forceinline__ void publish(gptr<float> p, float v) {
    __hip_atomic_store((float *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish(gptr<int32_t> p, int32_t v) {
    __hip_atomic_store((int32_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float fetch(gptr<float> p) {
    return __hip_atomic_load((float *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t fetch(gptr<int32_t> p) {
    return __hip_atomic_load((int32_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cluster barrier: every thread's published stores complete, thread 0 arrives and waits
// for the cluster with a bounded spin; on a timeout (or another cluster's abort) it raises
// the abort flag and every waiting workgroup leaves, so the grid always drains. Returns
// false on abort.
constexpr unsigned kSpinLimit = 1u << 22;

template <bool kNoPoll>
__device__ __forceinline__ bool cluster_sync(gptr<int32_t> bar_g, int target, int32_t *abort_flag) {
    int32_t *bar = (int32_t *)bar_g;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);   // this thread's published stores have completed
    __syncthreads();
    int ok = 1;
    if (threadIdx.x == 0) {
        auto wait_all = [&]() {
            unsigned spins = 0;
            while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
                if (++spins > kSpinLimit) {
                    atomicExch(abort_flag, 1);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        };
        if constexpr (kNoPoll) {
            // the last to arrive sees the full count in the add's own result and does not
            // poll (kept to the kernels whose registers leave room for it)
            if (__hip_atomic_fetch_add(bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 < target) wait_all();
        } else {
            __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wait_all();
        }
    }
    const bool all = __syncthreads_and(ok) != 0;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return all;
}

// Sum of the cluster's k partial gradients into g[0..nm) in rank order (every rank gets the
// same bits); returns the sum of the partial objectives.
__device__ __forceinline__ float read_partials(float *g, gptr<float> buf, int64_t pstride, int nm, int k) {
    for (int i = threadIdx.x; i < nm; i += blockDim.x) {
        float s = 0.0f;
        for (int q = 0; q < k; ++q) s += fetch(buf + (int64_t)q * pstride + i);
        g[i] = s;
    }
    float os = 0.0f;
    for (int q = 0; q < k; ++q) os += fetch(buf + (int64_t)q * pstride + nm);
    return os;
}

// The same for k = 2 with every load of a thread in flight before the first sum: one round
// trip to the coherence point instead of one per element (same sums, same order).
__device__ __forceinline__ float read_partials2(float *g, gptr<float> buf, int64_t pstride, int nm) {
    constexpr int kB = 4;
    const float o0 = fetch(buf + nm), o1 = fetch(buf + pstride + nm);
    for (int i0 = threadIdx.x; i0 < nm; i0 += kB * blockDim.x) {
        float v0[kB], v1[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            v0[u] = v1[u] = 0.0f;
            if (i < nm) {
                v0[u] = fetch(buf + i);
                v1[u] = fetch(buf + pstride + i);
            }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < nm) g[i] = (0.0f + v0[u]) + v1[u];
        }
    }
    return (0.0f + o0) + o1;
}

// Waves per workgroup of the solver kernel for each message variant: register-resident
// messages of the medium bound take about 200 VGPRs (8 waves per workgroup), those of the
// large bound all 256 (one wave per SIMD, 4 waves per workgroup).
template <int V> struct SolveWaves { static constexpr int value = 16; };
template <> struct SolveWaves<kMsgMedium> { static constexpr int value = 8; };
template <> struct SolveWaves<kMsgLarge> { static constexpr int value = 4; };

// kCluster: k workgroups per restart (k read from the descriptor); otherwise k = 1 and the
// kernel carries none of the cluster's exchange state.
template <int V, bool kCluster, bool kPair>
__global__ void __launch_bounds__(64 * SolveWaves<V>::value)
    solve_wg_kernel(const InstDesc *insts, SolveParams P, int32_t *stop_flags, int32_t *abort_flag) {
    using Ms = typename MsgOf<V>::type;
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int ii = find_inst(insts, P.n_inst, blockIdx.x);
    const InstDesc &I = insts[ii];
    const TabView T = I.T;
    const HalfSpaces hs = I.hs;
    const int k = kCluster ? I.k : 1;
    const int local = blockIdx.x - I.wg_base;
    const int r = local / k, rank = local - r * k;
    const int n = T.n_bool, m = T.n_real, C = T.n_cons;
    const int nw = (C + 31) >> 5;
    float *sa = lds, *sb = sa + n, *ga = sb + m, *gb = ga + n, *pb = gb + m, *ph = pb + m;
    const int NN = P.lds_nodes + 2, SS = P.lds_slots;
    FSMT_MSG_STORE(Ms, W, lds + P.state_floats + (size_t)wave * (2 * NN + 4 * SS) * 64, NN, SS, lane);
    const gptr<float> wrow = I.w + (int64_t)r * C, hrow = I.hist + (int64_t)r * C;
    // the ERWA weights are written by rank 0 at the end of a level and read by every rank's
    // sweep: in a cluster they go through the coherence point like the partials
    auto wload = [&](int c) -> float { return kCluster ? fetch(wrow + c) : (float)wrow[c]; };
    auto wstore = [&](int c, float v) {
        if (kCluster) publish(wrow + c, v); else wrow[c] = v;
    };
    const gptr<uint32_t> brow = I.sat_bits + (int64_t)r * nw;
    const int64_t pstride = (int64_t)n + m + 1;
    // partials and level results are double-buffered by exchange parity: a rank may publish
    // the next exchange while another is still reading this one, but it cannot get two
    // exchanges ahead (the barrier in between waits for every rank)
    const gptr<float> prow = kCluster ? I.part + (int64_t)r * 2 * k * pstride : nullptr;
    int xpar = 0, lpar = 0;
    int bar_target = 0;

    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        sa[i] = I.a[(int64_t)r * I.a_sr + i];
        ga[i] = 0.0f;
    }
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        sb[j] = I.b[(int64_t)r * I.b_sr + j];
        gb[j] = 0.0f;
    }
    int level = I.level_done[r];
    int steps_done = I.steps_done[r];
    int verdict = I.verdict[r];
    int n_unsat = I.n_unsat[r];
    float obj = I.obj[r];
    bool aborted = false;
    __syncthreads();
    const LdsState st{sa, sb};
    const LdsScatter sc{ga, gb};
    const int n_tasks = T.n_pos >> 6;

    while (level < P.n_levels && !(verdict == 1 && P.stop_mode != 0)) {
        const double kappa = P.kappas[level];
        const bool hard = isinf(kappa);
        for (int step = 0; step < P.steps; ++step) {
            // gradients are zero here: zeroed at entry and by the previous step's update
            float oacc = 0.0f;
            for (int task = rank + k * wave; task < n_tasks; task += k * P.waves) {
                const TaskCtx t = task_ctx(T, task * 64 + lane, r, true);
                const float wc = t.valid ? wload(t.c) : 0.0f;   // requested before the forward pass
                oacc += wc * task_eval<true, kPair>(T, t, st, kappa, hard, wc, sc, W, lane);
            }
            if (kCluster) {
                // publish this workgroup's partial gradient and objective, then sum the
                // cluster's partials in rank order (every rank gets the same bits)
                const float op = block_sum(oacc);
                const gptr<float> buf = prow + (int64_t)xpar * k * pstride;
                xpar ^= 1;
                const gptr<float> mine = buf + (int64_t)rank * pstride;
                for (int i = threadIdx.x; i < n + m; i += blockDim.x) publish(mine + i, ga[i]);
                if (threadIdx.x == 0) publish(mine + n + m, op);
                bar_target += k;
                if (!cluster_sync<V == kMsgSmall>(I.bar + r, bar_target, abort_flag)) {
                    aborted = true;
                    break;
                }
                float os;
                if constexpr (V == kMsgSmall) {
                    os = k == 2 ? read_partials2(ga, buf, pstride, n + m) : read_partials(ga, buf, pstride, n + m, k);
                } else {
                    os = read_partials(ga, buf, pstride, n + m, k);
                }
                oacc = threadIdx.x == 0 ? os : 0.0f;
            }
            __syncthreads();
            // projected step (Eq. pg1/pg2) and the gradient map norm (Eq. grad_map)
            float acc = 0.0f;
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const float x = sa[i], y = x - P.eta_a * ga[i];
                const float p = y < -1.0f ? -1.0f : (y > 1.0f ? 1.0f : y);
                sa[i] = p;
                ga[i] = 0.0f;
                const float g = (x - p) / P.eta_a;
                acc += g * g;
            }
            if (hs.n == 0) {
                for (int j = threadIdx.x; j < m; j += blockDim.x) {
                    const float x = sb[j], y = x - P.eta_b * gb[j];
                    const float p = y < T.real_lo[j] ? T.real_lo[j] : (y > T.real_hi[j] ? T.real_hi[j] : y);
                    sb[j] = p;
                    gb[j] = 0.0f;
                    const float g = (x - p) / P.eta_b;
                    acc += g * g;
                }
            } else {
                for (int j = threadIdx.x; j < m; j += blockDim.x) gb[j] = sb[j] - P.eta_b * gb[j];
                project_dykstra(gb, pb, ph, T.real_lo, T.real_hi, m, hs);
                for (int j = threadIdx.x; j < m; j += blockDim.x) {
                    const float x = sb[j], p = gb[j];
                    sb[j] = p;
                    gb[j] = 0.0f;
                    const float g = (x - p) / P.eta_b;
                    acc += g * g;
                }
            }
            const float2 red = block_sum2(oacc, acc);   // also orders the updates before the next sweep
            obj = red.x;
            ++steps_done;
            if (red.y <= P.eps2) break;
        }
        if (aborted) break;
        // rounding, exact check and ERWA (Alg. "CLS with Annealing"): rank 0 of the cluster
        int stop = 0;
        if (rank == 0) {
            const bool update = ((level + 1) % P.tau) == 0;
            float nu_acc = 0.0f, wsum = 0.0f;
            for (int c0 = wave * 64; c0 < C; c0 += P.waves * 64) {
                const int c = c0 + lane;
                const bool sat = c < C ? walk_state(T, st, c, r) : false;
                const uint64_t mask = __ballot(sat);
                if (lane == 0) {
                    brow[c0 >> 5] = (uint32_t)mask;
                    if ((c0 >> 5) + 1 < nw) brow[(c0 >> 5) + 1] = (uint32_t)(mask >> 32);
                }
                if (c < C) {
                    const float viol = sat ? 0.0f : 1.0f;
                    float h = P.rho * hrow[c] + viol;
                    float wv = wload(c);
                    if (update) {
                        wv *= powf(P.gamma, h);
                        h = 1.0f;
                        wstore(c, wv);
                    }
                    hrow[c] = h;
                    wsum += wv;
                    nu_acc += viol;
                }
            }
            n_unsat = (int)block_sum(nu_acc);
            if (update && P.normalize) {
                const float ws = block_sum(wsum);
                const float scale = (float)C / ws;
                for (int c = threadIdx.x; c < C; c += blockDim.x) wstore(c, wload(c) * scale);
            }
            if (n_unsat == 0 && P.stop_mode == 2 && threadIdx.x == 0) atomicExch(stop_flags + ii, 1);
            stop = (P.stop_mode == 2 && __syncthreads_or(threadIdx.x == 0 && atomicAdd(stop_flags + ii, 0) != 0)) ? 1 : 0;
            if (kCluster && threadIdx.x == 0) {
                publish(I.ctl + 4 * r + 2 * lpar, n_unsat);
                publish(I.ctl + 4 * r + 2 * lpar + 1, stop);
            }
        }
        if (kCluster) {
            bar_target += k;
            if (!cluster_sync<V == kMsgSmall>(I.bar + r, bar_target, abort_flag)) {
                aborted = true;
                break;
            }
            n_unsat = fetch(I.ctl + 4 * r + 2 * lpar);
            stop = fetch(I.ctl + 4 * r + 2 * lpar + 1);
            lpar ^= 1;
        }
        ++level;
        if (n_unsat == 0) verdict = 1;
        if (stop) break;
        __syncthreads();
    }
    __syncthreads();
    if (rank != 0) return;
    if (!aborted) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) I.a[(int64_t)r * I.a_sr + i] = sa[i];
        for (int j = threadIdx.x; j < m; j += blockDim.x) I.b[(int64_t)r * I.b_sr + j] = sb[j];
    }
    if (threadIdx.x == 0) {
        I.level_done[r] = level;
        I.steps_done[r] = steps_done;
        I.verdict[r] = aborted ? -2 : verdict;
        I.n_unsat[r] = n_unsat;
        I.obj[r] = obj;
    }
}

static fsmt_status launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FSMT_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FSMT_OK;
}

template <int V, bool kPair>
static const void *solve_kernel_fn_v(bool cl) {
    return cl ? (const void *)solve_wg_kernel<V, true, kPair> : (const void *)solve_wg_kernel<V, false, kPair>;
}
template <bool kPair>
static const void *solve_kernel_fn_p(int msg, bool cl) {
    if (msg == kMsgSmall) return solve_kernel_fn_v<kMsgSmall, kPair>(cl);
    if (msg == kMsgMedium) return solve_kernel_fn_v<kMsgMedium, kPair>(cl);
    if (msg == kMsgLarge) return solve_kernel_fn_v<kMsgLarge, kPair>(cl);
    return solve_kernel_fn_v<kMsgLds, kPair>(cl);
}
// The persistent solver kernel for a message variant, cluster mode and pair-disjunction path.
static const void *solve_kernel_fn(int msg, bool cl, bool pair) {
    return pair ? solve_kernel_fn_p<true>(msg, cl) : solve_kernel_fn_p<false>(msg, cl);
}

static int lds_budget_bytes() {
    static int budget = -1;
    if (budget < 0) {
        budget = 65536;
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > budget)
            budget = v;
        std::vector<const void *> fns;
        for (int msg : {kMsgLds, kMsgSmall, kMsgMedium, kMsgLarge})
            for (int cl = 0; cl < 2; ++cl)
                for (int pair = 0; pair < 2; ++pair) fns.push_back(solve_kernel_fn(msg, cl != 0, pair != 0));
        for (const void *f : fns) {
            if (budget > 65536 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, budget) != hipSuccess) {
                (void)hipGetLastError();
                budget = 65536;
            }
        }
    }
    return budget;
}

static int solve_waves(int msg) {
    return msg == kMsgMedium  ? SolveWaves<kMsgMedium>::value
           : msg == kMsgLarge ? SolveWaves<kMsgLarge>::value
                              : SolveWaves<kMsgSmall>::value;
}

static size_t state_floats_of(const fsmt_xbdd *h) {
    size_t f = 2 * (size_t)h->n_bool + 2 * (size_t)h->n_real;
    if (h->n_hs) f += (size_t)h->n_real + (size_t)h->hs_nnz;
    return (f + 63) / 64 * 64;
}

}  // namespace fsmt

using namespace fsmt;

// Schedule choice per instance (cost model in units of one wave task): the persistent
// schedule needs the restart's state in LDS and costs ceil(tasks / waves) sequential tasks
// per step on one CU; the grid schedule spreads tasks x restarts over all CUs (about 8 waves
// each) and pays two launches per step (about 20 task-times).
static bool prefer_grid(const fsmt_xbdd *h, int R, int64_t R_batch, int waves_a, int n_cu) {
    // persistent: a restart's tasks over its cluster of k workgroups (k as chosen below, with
    // every restart of the batch resident at once), plus the exchange of k partial
    // gradients per step
    const double tasks_a = (double)h->n_pos / 64.0;                  // per restart, lane = constraint
    const int wa = std::max(1, waves_a);
    int k = 1;
    while (k < 16 && tasks_a >= 2.0 * (2 * k) * wa && R_batch * 2 * k <= n_cu) k *= 2;
    const double exchange = k > 1 ? 4.0 + (double)(h->n_bool + h->n_real) * k / (wa * 64.0 * 16.0) : 0.0;
    const double t_a = std::ceil(tasks_a / (wa * k)) + exchange;
    // grid: every (constraint, restart) lane over the device, as many waves per CU as the
    // message store's registers allow, plus the launches of a step
    int rp = 1;
    while (rp < R && rp < 64) rp <<= 1;
    const double lanes = (double)h->n_pos * (R <= 64 ? rp : std::ceil(R / 64.0) * 64.0);
    const double t_b = std::ceil(lanes / 64.0 / ((double)wa * n_cu)) + 20.0;
    return t_b < t_a;
}

extern "C" fsmt_status fsmt_solve_batched(const fsmt_xbdd *const *insts, int32_t n_inst, const fsmt_solve_opts *opts,
                                          const fsmt_solve_state *states, void *stream) {
    clear_error();
    if (!insts || !opts || !states || n_inst <= 0) return set_error(FSMT_EINVAL, "null argument or no instance");
    const fsmt_solve_opts &O = *opts;
    if (O.n_levels < 0 || O.n_levels > kMaxLevels) return set_error(FSMT_ELIMIT, "n_levels must be in [0, %d]", kMaxLevels);
    if (O.n_levels > 0 && !O.kappas) return set_error(FSMT_EINVAL, "kappas is NULL");
    if (O.steps_per_level < 0) return set_error(FSMT_EINVAL, "steps_per_level < 0");
    if (!(O.eta_a > 0.0f) || !(O.eta_b > 0.0f)) return set_error(FSMT_EINVAL, "step sizes must be positive");
    if (O.tau < 1) return set_error(FSMT_EINVAL, "tau must be >= 1");
    if (!(O.gamma > 0.0f) || !(O.rho >= 0.0f)) return set_error(FSMT_EINVAL, "bad ERWA parameters");
    if (O.schedule < 0 || O.schedule > 2) return set_error(FSMT_EINVAL, "schedule %d unknown", O.schedule);
    if (O.stop_on_sat < 0 || O.stop_on_sat > 2) return set_error(FSMT_EINVAL, "stop_on_sat must be 0, 1 or 2");
    for (int t = 0; t < O.n_levels; ++t)
        if (!(O.kappas[t] >= 0.0)) return set_error(FSMT_EINVAL, "kappa[%d] must be in [0, +inf]", t);

    // ---- validate states, collect shapes
    int device = -1;
    fsmt_status rc;
    for (int i = 0; i < n_inst; ++i) {
        const fsmt_xbdd *h = insts[i];
        const fsmt_solve_state &S = states[i];
        if (!h) return set_error(FSMT_EINVAL, "instance %d: null handle", i);
        if ((rc = select_device(h))) return rc;
        if (device >= 0 && h->device != device) return set_error(FSMT_EINVAL, "instances on different devices");
        device = h->device;
        const int R = S.a.rows;
        if (R <= 0) return set_error(FSMT_EINVAL, "instance %d: no restarts", i);
        if (S.a.cols != h->n_bool || S.b.rows != R || S.b.cols != h->n_real)
            return set_error(FSMT_EINVAL, "instance %d: state shape does not match the instance", i);
        if ((h->n_bool > 1 && S.a.stride_v != 1) || (h->n_real > 1 && S.b.stride_v != 1) ||
            (R > 1 && ((h->n_bool > 0 && S.a.stride_r < h->n_bool) || (h->n_real > 0 && S.b.stride_r < h->n_real))))
            return set_error(FSMT_EINVAL, "instance %d: a and b must be row-major [R][n] with unit column stride", i);
        const void *ptrs[] = {h->n_bool ? S.a.data : nullptr, h->n_real ? S.b.data : nullptr, S.w, S.hist,
                              S.sat_bits, S.n_unsat, S.verdict, S.level_done, S.steps_done, S.obj, S.grad_a, S.grad_b};
        for (int q = 0; q < 12; ++q) {
            if (!ptrs[q] && q >= 2 && q < 10) return set_error(FSMT_EINVAL, "instance %d: state pointer %d is NULL", i, q);
            if ((rc = check_device_ptr(ptrs[q], h->device, "state"))) return rc;
        }
    }

    // ---- persistent-schedule geometry (max over its instances) and schedule choice
    const size_t budget = (size_t)lds_budget_bytes();
    int n_cu = 256;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    std::vector<char> use_grid(n_inst, 0);
    int64_t r_batch = 0;
    for (int i = 0; i < n_inst; ++i) r_batch += states[i].a.rows;
    for (int i = 0; i < n_inst; ++i) {
        const fsmt_xbdd *h = insts[i];
        const int mv = msg_variant(h->small_max_nodes, h->small_max_slots, lds_store(h), h->all_inline);
        const size_t wb = mv == kMsgLds ? WaveScratch::bytes(h->small_max_nodes + 2, std::max(h->small_max_slots, 1)) : 0;
        const size_t sb = state_floats_of(h) * sizeof(float);
        const bool fits = sb + wb <= budget;
        const int waves = !fits ? 0 : wb ? (int)std::min<size_t>(16, (budget - sb) / wb) : solve_waves(mv);
        if (O.schedule == 1 && !fits)
            return set_error(FSMT_EUNSUPPORTED, "instance %d: restart state (%zu B) does not fit the persistent "
                             "schedule's LDS (%zu B)", i, sb, budget);
        // big diagrams are evaluated level by level by their own kernel, in the grid schedule
        if (O.schedule == 1 && h->n_big > 0)
            return set_error(FSMT_EUNSUPPORTED, "instance %d: %d big diagrams need the grid schedule", i, h->n_big);
        use_grid[i] = O.schedule == 2 || !fits || h->n_big > 0 ||
                      (O.schedule == 0 && prefer_grid(h, states[i].a.rows, r_batch, waves, n_cu));
    }

    hipStream_t st = (hipStream_t)stream;
    std::vector<int> ia, ib;
    for (int i = 0; i < n_inst; ++i) (use_grid[i] ? ib : ia).push_back(i);

    // the grid part runs on a forked stream, concurrently with the persistent launch
    hipStream_t gst = st;
    hipEvent_t fork = nullptr, join = nullptr;
    if (!ia.empty() && !ib.empty()) {
        if (hipStreamCreateWithFlags(&gst, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess)
            return set_error(FSMT_EHIP, "stream / event creation failed");
        (void)hipEventRecord(fork, st);
        (void)hipStreamWaitEvent(gst, fork, 0);
    }

    rc = FSMT_OK;
    // ---- persistent schedule
    if (!ia.empty()) {
        SolveParams P{};
        P.n_inst = (int)ia.size();
        P.n_levels = O.n_levels;
        P.steps = O.steps_per_level;
        P.tau = O.tau;
        P.normalize = O.normalize ? 1 : 0;
        P.stop_mode = O.stop_on_sat;
        P.eta_a = O.eta_a;
        P.eta_b = O.eta_b;
        P.eps2 = O.eps > 0.0f ? O.eps * O.eps : -1.0f;
        P.rho = O.rho;
        P.gamma = O.gamma;
        for (int t = 0; t < O.n_levels; ++t) P.kappas[t] = O.kappas[t];
        std::vector<InstDesc> desc(ia.size());
        size_t state_f = 0;
        int maxn = 0, maxs = 1;
        int64_t total_r = 0, min_tasks = INT64_MAX, part_floats = 0;
        for (size_t q = 0; q < ia.size(); ++q) {
            const fsmt_xbdd *h = insts[ia[q]];
            state_f = std::max(state_f, state_floats_of(h));
            maxn = std::max(maxn, h->small_max_nodes);
            maxs = std::max(maxs, h->small_max_slots);
            total_r += states[ia[q]].a.rows;
            min_tasks = std::min<int64_t>(min_tasks, h->n_pos / 64);
        }
        bool lds_only = false, all_inline = true;
        for (size_t q = 0; q < ia.size(); ++q) {
            lds_only = lds_only || lds_store(insts[ia[q]]);
            all_inline = all_inline && insts[ia[q]]->all_inline;
        }
        const int msg = msg_variant(maxn, maxs, lds_only, all_inline);
        const size_t wave_bytes = msg == kMsgLds ? WaveScratch::bytes(maxn + 2, maxs) : 0;
        const size_t state_bytes = state_f * sizeof(float);
        const int waves = wave_bytes ? (int)std::min<size_t>(16, (budget - state_bytes) / wave_bytes) : solve_waves(msg);
        const size_t lds = state_bytes + (size_t)waves * wave_bytes;
        // the cluster kernels (k workgroups per restart) have their own resource use
        bool pair = false;
        for (size_t q = 0; q < ia.size(); ++q) pair = pair || insts[ia[q]]->n_pair > 0;
        auto kernel_of = [&](bool cl) -> const void * { return solve_kernel_fn(msg, cl, pair); };
        auto resident_of = [&](bool cl) -> int64_t {
            int occ = 1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel_of(cl), 64 * waves, lds) != hipSuccess) {
                (void)hipGetLastError();
                occ = 1;
            }
            return (int64_t)n_cu * std::max(occ, 1);
        };
        // workgroups per restart: a cluster of k co-resident workgroups shares one restart's
        // sweep (all of them must be resident at once: their barrier waits for each other)
        int k = 1;
        if (O.cluster > 0) {
            k = O.cluster;
            if (k > 16 || (k > 1 && (total_r * k > resident_of(true) || !ib.empty())))
                return set_error(FSMT_EUNSUPPORTED, "cluster of %d workgroups per restart cannot be co-resident", k);
        } else if (ib.empty()) {
            // automatic: the largest power of two that leaves each wave at least two tasks
            // per step and keeps every workgroup resident. Measured per PGD step: config 3
            // (182 tasks per restart, 8 waves), 16 restarts: 306 us at k = 1, 163 at 2, 89 at
            // 4, 59 at 8; config 2 (66 tasks, 16 waves), 64 restarts: 22.8 us at k = 1,
            // 21.9 at 2, 22.9 at 4.
            const int64_t res = resident_of(true);
            while (k < 16 && min_tasks >= (int64_t)2 * (2 * k) * waves && total_r * 2 * k <= res) k *= 2;
        }
        const bool cl = k > 1;
        int64_t wg = 0;
        for (size_t q = 0; q < ia.size(); ++q) {
            const fsmt_xbdd *h = insts[ia[q]];
            const fsmt_solve_state &S = states[ia[q]];
            InstDesc &d = desc[q];
            d.T = TabView::of(h);
            d.hs = halfspaces_of(h);
            d.a = as_gptr(S.a.data);
            d.b = as_gptr(S.b.data);
            d.a_sr = S.a.stride_r;
            d.b_sr = S.b.stride_r;
            d.w = as_gptr(S.w);
            d.hist = as_gptr(S.hist);
            d.sat_bits = as_gptr(S.sat_bits);
            d.n_unsat = as_gptr(S.n_unsat);
            d.verdict = as_gptr(S.verdict);
            d.level_done = as_gptr(S.level_done);
            d.steps_done = as_gptr(S.steps_done);
            d.obj = as_gptr(S.obj);
            d.R = S.a.rows;
            d.k = k;
            d.wg_base = (int32_t)wg;
            wg += (int64_t)d.R * k;
            if (k > 1) part_floats += (int64_t)d.R * 2 * k * ((int64_t)h->n_bool + h->n_real + 1);
        }
        if (wg > INT32_MAX) return set_error(FSMT_ELIMIT, "too many restarts");
        P.lds_nodes = maxn;
        P.lds_slots = maxs;
        P.state_floats = (int32_t)state_f;
        P.waves = waves;
        // scratch: descriptors | stop flags [n] | abort flag | barriers [R] | level results [2][2R] | partials [2]
        void *dbuf = nullptr;
        const size_t desc_bytes = sizeof(InstDesc) * desc.size();
        const size_t off_flag = (desc_bytes + 255) / 256 * 256;
        const size_t n_int = desc.size() + 1 + 5 * (size_t)total_r;
        const size_t off_part = off_flag + (n_int * sizeof(int32_t) + 255) / 256 * 256;
        if (hipMallocAsync(&dbuf, off_part + sizeof(float) * (size_t)part_floats + 256, st) != hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(FSMT_ENOMEM, "descriptor allocation failed");
        } else {
            int32_t *ints = (int32_t *)((char *)dbuf + off_flag);
            int32_t *flags = ints, *abort_flag = ints + desc.size(), *bar = abort_flag + 1, *ctl = bar + total_r;
            float *part = (float *)((char *)dbuf + off_part);
            int64_t rb = 0, pb = 0;
            for (InstDesc &d : desc) {
                d.bar = as_gptr(bar + rb);
                d.ctl = as_gptr(ctl + 4 * rb);
                d.part = k > 1 ? as_gptr(part + pb) : nullptr;
                rb += d.R;
                if (k > 1) pb += (int64_t)d.R * 2 * k * ((int64_t)d.T.n_bool + d.T.n_real + 1);
            }
            if (hipMemcpyAsync(dbuf, desc.data(), desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
                fill_i32(ints, (int64_t)n_int, 0, st) != FSMT_OK) {
                rc = set_error(FSMT_EHIP, "descriptor upload failed");
            } else {
                const dim3 g((unsigned)wg), b(64 * waves);
                const InstDesc *d = (const InstDesc *)dbuf;
                void *args[] = {(void *)&d, (void *)&P, (void *)&flags, (void *)&abort_flag};
                const hipError_t le = hipLaunchKernel(kernel_of(k > 1), g, b, args, lds, st);
                rc = le != hipSuccess ? set_error(FSMT_EHIP, "solver kernel: %s", hipGetErrorString(le))
                                      : launch_status("solver kernel");
            }
            (void)hipFreeAsync(dbuf, st);
        }
    }

    // ---- grid schedule
    if (!ib.empty() && !rc) {
        std::vector<GridInst> gi(ib.size());
        int total_r = 0;
        int64_t tasks = 0, checks = 0, scratch_floats = 0, level_tasks = 0, big_restarts = 0;
        int lvl_nodes = 0, lvl_slots = 1;
        int maxn = 0, maxs = 1;
        size_t step_lds = 0;
        for (size_t q = 0; q < ib.size(); ++q) {
            const fsmt_xbdd *h = insts[ib[q]];
            const fsmt_solve_state &S = states[ib[q]];
            GridInst &d = gi[q];
            d.T = TabView::of(h);
            d.hs = halfspaces_of(h);
            d.a = as_gptr(S.a.data);
            d.b = as_gptr(S.b.data);
            d.a_sr = S.a.stride_r;
            d.b_sr = S.b.stride_r;
            d.ga = as_gptr(S.grad_a);
            d.gb = as_gptr(S.grad_b);
            d.ga_sr = h->n_bool;
            d.gb_sr = h->n_real;
            d.w = as_gptr(S.w);
            d.hist = as_gptr(S.hist);
            d.sat_bits = as_gptr(S.sat_bits);
            d.n_unsat = as_gptr(S.n_unsat);
            d.verdict = as_gptr(S.verdict);
            d.level_done = as_gptr(S.level_done);
            d.steps_done = as_gptr(S.steps_done);
            d.obj = as_gptr(S.obj);
            d.R = S.a.rows;
            int rp = 1, lg = 0;
            while (rp < d.R && rp < 64) { rp <<= 1; ++lg; }
            d.R_pad = d.R <= 64 ? rp : (d.R + 63) / 64 * 64;
            d.log2_rpad = d.R <= 64 ? lg : 0;
            d.rbase = total_r;
            d.task_base = tasks;
            d.check_base = checks;
            d.lev = as_cptr(h->d.lev);
            d.big_pos = as_cptr(h->d.big_pos);
            d.n_big = h->n_big;
            d.pad = 0;
            big_restarts += (int64_t)h->n_big * d.R;
            if (h->n_big > 0) {
                lvl_nodes = std::max(lvl_nodes, h->big_max_nodes);
                lvl_slots = std::max(lvl_slots, h->big_max_slots);
            }
            total_r += d.R;
            tasks += d.R <= 64 ? (int64_t)h->n_pos * d.R_pad / 64 : (int64_t)h->n_pos * (d.R_pad / 64);
            checks += (int64_t)d.R * ((h->n_cons + 255) / 256);
            if (!S.grad_a || !S.grad_b) scratch_floats += (int64_t)d.R * (h->n_bool + h->n_real);
            maxn = std::max(maxn, h->small_max_nodes);
            maxs = std::max(maxs, h->small_max_slots);
            if (h->n_hs) step_lds = std::max(step_lds, (size_t)(2 * h->n_real + h->hs_nnz) * sizeof(float));
        }
        bool lds_only = false, all_inline = true;
        for (size_t q = 0; q < ib.size(); ++q) {
            lds_only = lds_only || lds_store(insts[ib[q]]);
            all_inline = all_inline && insts[ib[q]]->all_inline;
        }
        const int msg = msg_variant(maxn, maxs, lds_only, all_inline);
        const size_t wave_bytes = msg == kMsgLds ? WaveScratch::bytes(maxn + 2, maxs) : 0;
        if (wave_bytes > 65536) rc = set_error(FSMT_ELIMIT, "diagram too large for the grid schedule");
        // level tasks: (big constraint, chunk of restarts), instance-major
        const int lvl_chunk = level_chunk(big_restarts, n_cu);
        for (GridInst &d : gi) {
            d.level_base = level_tasks;
            level_tasks += (int64_t)d.n_big * ((d.R + lvl_chunk - 1) / lvl_chunk);
        }
        const size_t level_bytes = level_tasks > 0 ? level_wave_floats(lvl_nodes, lvl_slots) * sizeof(float) : 0;
        if (level_bytes > 65536) rc = set_error(FSMT_ELIMIT, "diagram too large for the level-synchronous pass");
        if (step_lds > 65536) rc = set_error(FSMT_ELIMIT, "projection work arrays exceed LDS");
        // device scratch: descriptors, kappas, per-restart flags and accumulators, gradients
        const size_t off_k = (sizeof(GridInst) * gi.size() + 255) / 256 * 256;
        const size_t off_act = off_k + (sizeof(double) * std::max(1, O.n_levels) + 255) / 256 * 256;
        const size_t off_stp = off_act + (sizeof(int32_t) * total_r + 255) / 256 * 256;
        const size_t off_obj = off_stp + (sizeof(int32_t) * total_r + 255) / 256 * 256;
        const size_t off_flg = off_obj + (sizeof(float) * total_r + 255) / 256 * 256;
        const size_t off_grd = off_flg + (sizeof(int32_t) * gi.size() + 255) / 256 * 256;
        const size_t total = off_grd + sizeof(float) * (size_t)scratch_floats + 256;
        void *buf = nullptr;
        if (!rc && hipMallocAsync(&buf, total, gst) != hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(FSMT_ENOMEM, "grid schedule scratch allocation failed");
        }
        if (!rc) {
            char *base = (char *)buf;
            float *grd = (float *)(base + off_grd);
            for (GridInst &d : gi) {
                if (!d.ga || !d.gb) {
                    d.ga = as_gptr(grd);
                    d.gb = as_gptr(grd + (int64_t)d.R * d.T.n_bool);
                    grd += (int64_t)d.R * (d.T.n_bool + d.T.n_real);
                }
            }
            GridShared S{};
            S.kappas = (const double *)(base + off_k);
            S.active = (int32_t *)(base + off_act);
            S.stepping = (int32_t *)(base + off_stp);
            S.obj_acc = (float *)(base + off_obj);
            S.stop_flags = (int32_t *)(base + off_flg);
            S.total_r = total_r;
            S.n_levels = O.n_levels;
            S.stop_mode = O.stop_on_sat;
            S.tau = O.tau;
            S.normalize = O.normalize ? 1 : 0;
            S.lds_nodes = maxn;
            S.lds_slots = maxs;
            S.eta_a = O.eta_a;
            S.eta_b = O.eta_b;
            S.eps2 = O.eps > 0.0f ? O.eps * O.eps : -1.0f;
            S.rho = O.rho;
            S.gamma = O.gamma;
            S.total_tasks = tasks;
            S.level_tasks = level_tasks;
            S.level_nodes = lvl_nodes;
            S.level_slots = lvl_slots;
            S.level_chunk = lvl_chunk;
            std::vector<double> kap(O.kappas, O.kappas + O.n_levels);
            if (hipMemcpyAsync(base, gi.data(), sizeof(GridInst) * gi.size(), hipMemcpyHostToDevice, gst) != hipSuccess ||
                (O.n_levels > 0 && hipMemcpyAsync(base + off_k, kap.data(), sizeof(double) * kap.size(),
                                                  hipMemcpyHostToDevice, gst) != hipSuccess) ||
                fill_i32(S.stop_flags, (int64_t)gi.size(), 0, gst) != FSMT_OK ||
                fill_f32((float *)(base + off_grd), scratch_floats, 0.0f, gst) != FSMT_OK) {
                rc = set_error(FSMT_EHIP, "grid schedule upload failed");
            } else {
                GridPlan plan{};
                plan.steps = O.steps_per_level;
                plan.msg = msg;
                plan.sweep_wpb = wave_bytes ? (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / wave_bytes)) : 4;
                plan.sweep_lds = wave_bytes * plan.sweep_wpb;
                plan.sweep_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((tasks + plan.sweep_wpb - 1) / plan.sweep_wpb,
                                                                               (int64_t)n_cu * 8));
                plan.step_lds = step_lds;
                plan.level_wpb = level_bytes ? (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / level_bytes)) : 1;
                plan.level_lds = level_bytes * plan.level_wpb;
                plan.level_blocks = level_tasks > 0 ? (int)std::min<int64_t>((level_tasks + plan.level_wpb - 1) / plan.level_wpb,
                                                                             (int64_t)n_cu * 16)
                                                    : 0;
                plan.check_blocks = checks;
                plan.use_graph = true;
                plan.pair = false;
                for (size_t q = 0; q < ib.size(); ++q) plan.pair = plan.pair || insts[ib[q]]->n_pair > 0;
                // replay only the levels some restart still has to run: a call that resumes a
                // schedule (level_done > 0) would otherwise replay every finished level as
                // launches with nothing to do
                int first = O.n_levels;
                for (size_t q = 0; q < ib.size() && !rc; ++q) {
                    const fsmt_solve_state &St = states[ib[q]];
                    const int R = St.a.rows;
                    std::vector<int32_t> lv((size_t)R), vd((size_t)R);
                    if (hipMemcpyAsync(lv.data(), St.level_done, sizeof(int32_t) * R, hipMemcpyDeviceToHost, gst) != hipSuccess ||
                        hipMemcpyAsync(vd.data(), St.verdict, sizeof(int32_t) * R, hipMemcpyDeviceToHost, gst) != hipSuccess ||
                        hipStreamSynchronize(gst) != hipSuccess) {
                        rc = set_error(FSMT_EHIP, "reading level counters failed");
                        break;
                    }
                    for (int r = 0; r < R; ++r)
                        if (!(vd[r] == 1 && O.stop_on_sat != 0)) first = std::min(first, std::max(lv[r], 0));
                }
                if (!rc) rc = run_grid_schedule((const GridInst *)buf, (int)gi.size(), S, plan, O.n_levels - first, gst);
            }
            (void)hipFreeAsync(buf, gst);
        }
    }

    if (join) {
        (void)hipEventRecord(join, gst);
        (void)hipStreamWaitEvent(st, join, 0);
        (void)hipStreamSynchronize(gst);
        (void)hipEventDestroy(fork);
        (void)hipEventDestroy(join);
        (void)hipStreamDestroy(gst);
    }
    return rc;
}
