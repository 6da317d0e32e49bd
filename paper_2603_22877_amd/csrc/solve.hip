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
#include <mutex>
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
    uint32_t spin_limit;    // polls of a cluster barrier before it gives up
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
__device__ __forceinline__ bool cluster_sync(gptr<int32_t> bar_g, int target, int32_t *abort_flag,
                                             unsigned spin_limit) {
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
                if (++spins > spin_limit) {
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
// same bits); returns the sum of the partial objectives. A thread issues the loads of kQ
// partials of kB elements before summing them, so such a batch costs one round trip to
// the coherence point (kernels with registers to spare take larger batches).
template <int kB, int kQ>
__device__ __forceinline__ float read_partials(float *g, gptr<float> buf, int64_t pstride, int nm, int k) {
    float os = 0.0f;
    for (int q0 = 0; q0 < k; q0 += kQ) {
        float v[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) v[q] = q0 + q < k ? fetch(buf + (int64_t)(q0 + q) * pstride + nm) : 0.0f;
#pragma unroll
        for (int q = 0; q < kQ; ++q)
            if (q0 + q < k) os += v[q];
    }
    for (int i0 = threadIdx.x; i0 < nm; i0 += kB * blockDim.x) {
        float s[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) s[u] = 0.0f;
        for (int q0 = 0; q0 < k; q0 += kQ) {
            float v[kB][kQ];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int i = i0 + u * (int)blockDim.x;
#pragma unroll
                for (int q = 0; q < kQ; ++q)
                    v[u][q] = (q0 + q < k && i < nm) ? fetch(buf + (int64_t)(q0 + q) * pstride + i) : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kB; ++u)
#pragma unroll
                for (int q = 0; q < kQ; ++q)
                    if (q0 + q < k) s[u] += v[u][q];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < nm) g[i] = s[u];
        }
    }
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

// Waves per workgroup of the solver kernel for each message variant and closed-form level:
// register-resident messages of the medium bound take about 200 VGPRs (8 waves per
// workgroup), those of the large bound all 256 (one wave per SIMD, 4 waves per workgroup);
// the closed forms of two selectors over eight atoms need more than the 128 VGPRs that 16
// waves leave: 12 waves (168 VGPRs; measured on placement 1,200 at 16 restarts, 369 us per
// PGD iteration against 458 us with 8 waves of 206 VGPRs, the spills being in the set-up).
template <int V, int kCF> struct SolveWaves { static constexpr int value = kCF >= 2 ? 12 : 16; };
template <int kCF> struct SolveWaves<kMsgMedium, kCF> { static constexpr int value = 8; };
template <int kCF> struct SolveWaves<kMsgLarge, kCF> { static constexpr int value = 4; };

// kCluster: k workgroups per restart (k read from the descriptor); otherwise k = 1 and the
// kernel carries none of the cluster's exchange state.
template <int V, bool kCluster, int kCF>
__global__ void __launch_bounds__((64 * SolveWaves<V, kCF>::value))
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
    int verdict = I.verdict[r] == 1 ? 1 : 0;   // -2 (an earlier call gave up) resumes as not SAT
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
                oacc += wc * task_eval<true, kCF>(T, t, st, kappa, hard, wc, sc, W, lane);
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
                if (!cluster_sync<V == kMsgSmall>(I.bar + r, bar_target, abort_flag, P.spin_limit)) {
                    aborted = true;
                    break;
                }
                float os;
                if constexpr (SolveWaves<V, kCF>::value >= 16) {   // 128 VGPRs: small batches
                    os = k == 2 ? read_partials2(ga, buf, pstride, n + m) : read_partials<1, 4>(ga, buf, pstride, n + m, k);
                } else {
                    os = read_partials<2, 16>(ga, buf, pstride, n + m, k);
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
        // rounding, exact check and ERWA (Alg. "CLS with Annealing"): every rank of the
        // cluster checks its share of the constraints (64-constraint blocks dealt round-robin
        // over ranks and waves). The violated counts and the sums of the updated weights are
        // exchanged like the partial gradients; only then does each rank store its share's new
        // history and (normalized) weights, recomputed from its check bits, so a cluster that
        // gives up at the exchange leaves the weights of the last completed level.
        int stop = 0;
        {
            const bool update = ((level + 1) % P.tau) == 0;
            auto erwa = [&](bool sat, float h0, float w0, float &h, float &wv) {
                h = P.rho * h0 + (sat ? 0.0f : 1.0f);
                wv = w0;
                if (update) {
                    wv *= powf(P.gamma, h);
                    h = 1.0f;
                }
            };
            float nu_acc = 0.0f, wsum = 0.0f;
            for (int c0 = (rank + k * wave) * 64; c0 < C; c0 += k * P.waves * 64) {
                const int c = c0 + lane;
                const bool sat = c < C ? walk_state(T, st, c, r) : false;
                const uint64_t mask = __ballot(sat);
                if (lane == 0) {
                    brow[c0 >> 5] = (uint32_t)mask;
                    if ((c0 >> 5) + 1 < nw) brow[(c0 >> 5) + 1] = (uint32_t)(mask >> 32);
                }
                if (c < C) {
                    float h, wv;
                    erwa(sat, hrow[c], wload(c), h, wv);
                    wsum += wv;
                    nu_acc += sat ? 0.0f : 1.0f;
                }
            }
            float2 tot = block_sum2(nu_acc, wsum);   // also orders the bit stores before the reads below
            if (kCluster) {
                const gptr<float> buf = prow + (int64_t)xpar * k * pstride;
                xpar ^= 1;
                if (threadIdx.x == 0) {
                    publish(buf + (int64_t)rank * pstride, tot.x);
                    publish(buf + (int64_t)rank * pstride + 1, tot.y);
                }
                bar_target += k;
                if (!cluster_sync<V == kMsgSmall>(I.bar + r, bar_target, abort_flag, P.spin_limit)) {
                    aborted = true;
                    break;
                }
                tot = make_float2(0.0f, 0.0f);
                for (int q = 0; q < k; ++q) {   // rank order: every rank gets the same sums
                    tot.x += fetch(buf + (int64_t)q * pstride);
                    tot.y += fetch(buf + (int64_t)q * pstride + 1);
                }
            }
            n_unsat = (int)tot.x;
            const float scale = (update && P.normalize) ? (float)C / tot.y : 1.0f;
            for (int c0 = (rank + k * wave) * 64; c0 < C; c0 += k * P.waves * 64) {
                const int c = c0 + lane;
                if (c < C) {
                    const bool sat = (brow[c >> 5] >> (c & 31)) & 1u;
                    float h, wv;
                    erwa(sat, hrow[c], wload(c), h, wv);
                    hrow[c] = h;
                    if (update) wstore(c, (update && P.normalize) ? wv * scale : wv);
                }
            }
            if (rank == 0) {
                if (n_unsat == 0 && P.stop_mode == 2 && threadIdx.x == 0) atomicExch(stop_flags + ii, 1);
                stop = (P.stop_mode == 2 && __syncthreads_or(threadIdx.x == 0 && atomicAdd(stop_flags + ii, 0) != 0)) ? 1 : 0;
                // the level is complete: its point and counters go to memory (the other ranks'
                // weights are stored before they reach the barrier below, so a call that ends
                // there leaves a state that a later call resumes consistently)
                for (int i = threadIdx.x; i < n; i += blockDim.x) I.a[(int64_t)r * I.a_sr + i] = sa[i];
                for (int j = threadIdx.x; j < m; j += blockDim.x) I.b[(int64_t)r * I.b_sr + j] = sb[j];
                if (threadIdx.x == 0) {
                    I.level_done[r] = level + 1;
                    I.steps_done[r] = steps_done;
                    I.n_unsat[r] = n_unsat;
                    I.obj[r] = obj;
                    I.verdict[r] = n_unsat == 0 ? 1 : verdict;
                }
                if (kCluster && threadIdx.x == 0) publish(I.ctl + 4 * r + 2 * lpar + 1, stop);
            }
        }
        if (aborted) break;
        if (kCluster) {
            bar_target += k;
            if (!cluster_sync<V == kMsgSmall>(I.bar + r, bar_target, abort_flag, P.spin_limit)) {
                aborted = true;
                break;
            }
            stop = fetch(I.ctl + 4 * r + 2 * lpar + 1);
            lpar ^= 1;
        }
        ++level;
        if (n_unsat == 0) verdict = 1;
        if (stop) break;
        __syncthreads();
    }
    // every completed level was written back at its end; an aborted restart only marks its
    // verdict (its state is that of its last completed level)
    if (aborted && rank == 0 && threadIdx.x == 0) I.verdict[r] = -2;
}

static fsmt_status launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FSMT_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FSMT_OK;
}

template <int V, int kCF>
static const void *solve_kernel_fn_v(bool cl) {
    return cl ? (const void *)solve_wg_kernel<V, true, kCF> : (const void *)solve_wg_kernel<V, false, kCF>;
}
template <int kCF>
static const void *solve_kernel_fn_p(int msg, bool cl) {
    if (msg == kMsgSmall) return solve_kernel_fn_v<kMsgSmall, kCF>(cl);
    if (msg == kMsgMedium) return solve_kernel_fn_v<kMsgMedium, kCF>(cl);
    if (msg == kMsgLarge) return solve_kernel_fn_v<kMsgLarge, kCF>(cl);
    return solve_kernel_fn_v<kMsgLds, kCF>(cl);
}
// The persistent solver kernel for a message variant, cluster mode and closed-form level.
static const void *solve_kernel_fn(int msg, bool cl, int cf) {
    return cf == 0 ? solve_kernel_fn_p<0>(msg, cl)
           : cf == 1 ? solve_kernel_fn_p<1>(msg, cl)
           : cf == 2 ? solve_kernel_fn_p<2>(msg, cl)
                     : solve_kernel_fn_p<3>(msg, cl);
}

// Dynamic LDS a persistent workgroup may take: the device's per-block maximum (opted into
// for every solver kernel) less the largest static LDS of those kernels (the block
// reductions' partial sums).
static int lds_budget_bytes() {
    static int budget = -1;
    if (budget < 0) {
        int b = 65536;
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > b)
            b = v;
        std::vector<const void *> fns;
        for (int msg : {kMsgLds, kMsgSmall, kMsgMedium, kMsgLarge})
            for (int cl = 0; cl < 2; ++cl)
                for (int cf = 0; cf < 4; ++cf) fns.push_back(solve_kernel_fn(msg, cl != 0, cf));
        size_t static_lds = 0;
        for (const void *f : fns) {
            hipFuncAttributes fa{};
            if (hipFuncGetAttributes(&fa, f) == hipSuccess) static_lds = std::max(static_lds, (size_t)fa.sharedSizeBytes);
            else (void)hipGetLastError();
        }
        const int dyn = b - (int)static_lds;
        for (const void *f : fns) {
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) {
                (void)hipGetLastError();
                b = 65536;
            }
        }
        budget = b - (int)static_lds;
    }
    return budget;
}

static int solve_waves(int msg, int cf) {
    if (msg == kMsgMedium) return SolveWaves<kMsgMedium, 0>::value;
    if (msg == kMsgLarge) return SolveWaves<kMsgLarge, 0>::value;
    return cf >= 2 ? SolveWaves<kMsgSmall, 2>::value : SolveWaves<kMsgSmall, 0>::value;
}

static size_t state_floats_of(const fsmt_xbdd *h) {
    size_t f = 2 * (size_t)h->n_bool + 2 * (size_t)h->n_real;
    if (h->n_hs) f += (size_t)h->n_real + (size_t)h->hs_nnz;
    return (f + 63) / 64 * 64;
}

// ---- per-device resources kept for the life of the process
// A stream for the grid part of a mixed batch, a stream to capture level graphs on, the
// fork/join events, and instantiated level graphs waiting for their last launch to finish
// before they are destroyed (checked without blocking at the next call).
constexpr int kMaxDevices = 64;
struct DeviceRes {
    bool init = false;
    hipStream_t fork = nullptr, cap = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<GraphRetired> retired;
};
static std::mutex g_res_mutex;
static DeviceRes g_res[kMaxDevices];

// Called with g_res_mutex held and `device` current.
static fsmt_status device_res(int device, DeviceRes **out) {
    if (device < 0 || device >= kMaxDevices) return set_error(FSMT_EINVAL, "device %d out of range", device);
    DeviceRes &R = g_res[device];
    if (!R.init) {
        if (hipStreamCreateWithFlags(&R.fork, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&R.cap, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&R.ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&R.ev_join, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FSMT_EHIP, "solver stream / event creation failed on device %d", device);
        }
        R.init = true;
    }
    reap_retired(R.retired);
    *out = &R;
    return FSMT_OK;
}

// Device memory of one call: either allocated stream-ordered on the call's stream (and
// freed the same way after the kernels), or carved from a fixed buffer (the allocation-free
// entry point).
struct CallScratch {
    char *fixed = nullptr;     // base of the fixed buffer, or null
    size_t cap = 0, used = 0;
    fsmt_status get(size_t bytes, hipStream_t st, void **out) {
        bytes = (bytes + 255) / 256 * 256;
        if (fixed) {
            if (used + bytes > cap)
                return set_error(FSMT_ELIMIT, "the call needs more than the %zu bytes of the fixed solver scratch", cap);
            *out = fixed + used;
            used += bytes;
            return FSMT_OK;
        }
        if (hipMallocAsync(out, bytes, st) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FSMT_ENOMEM, "solver scratch allocation (%zu bytes) failed", bytes);
        }
        return FSMT_OK;
    }
    void put(void *p, hipStream_t st) const {
        if (!fixed && p) (void)hipFreeAsync(p, st);
    }
};

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

// Geometry of one persistent launch over a set of instances.
struct PersistentGeom {
    int msg = kMsgSmall, waves = 0, maxn = 0, maxs = 1;
    size_t state_f = 0, wave_bytes = 0, lds = 0;
    int cf = 0;
};

static PersistentGeom persistent_geom(const fsmt_xbdd *const *insts, const std::vector<int> &ids, size_t budget) {
    PersistentGeom G;
    bool lds_only = false, all_inline = true;
    for (int i : ids) {
        const fsmt_xbdd *h = insts[i];
        G.state_f = std::max(G.state_f, state_floats_of(h));
        G.maxn = std::max(G.maxn, h->small_max_nodes);
        G.maxs = std::max(G.maxs, h->small_max_slots);
        lds_only = lds_only || lds_store(h);
        all_inline = all_inline && h->all_inline;
        G.cf = std::max(G.cf, closed_level(h));
    }
    G.msg = msg_variant(G.maxn, G.maxs, lds_only, all_inline);
    G.wave_bytes = G.msg == kMsgLds ? WaveScratch::bytes(G.maxn + 2, G.maxs) : 0;
    const size_t state_bytes = G.state_f * sizeof(float);
    if (state_bytes > budget) {
        G.waves = 0;
    } else if (G.wave_bytes) {
        G.waves = (int)std::min<size_t>(solve_waves(G.msg, G.cf), (budget - state_bytes) / G.wave_bytes);
    } else {
        G.waves = solve_waves(G.msg, G.cf);
    }
    G.lds = state_bytes + (size_t)G.waves * G.wave_bytes;
    return G;
}

namespace fsmt {

fsmt_status solve_impl(const fsmt_xbdd *const *insts, int32_t n_inst, const fsmt_solve_opts *opts,
                       const fsmt_solve_state *states, void *stream, void *fixed, size_t fixed_cap) {
    const bool fixed_scratch = fixed != nullptr;
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
    if (O.level_begin < 0) return set_error(FSMT_EINVAL, "level_begin < 0");
    if (O.spin_limit < 0) return set_error(FSMT_EINVAL, "spin_limit < 0");
    if (fixed_scratch && O.schedule == 2) return set_error(FSMT_EUNSUPPORTED, "the allocation-free call runs the persistent schedule only");
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

    // the device's streams, events and retired graphs serve the grid schedule and mixed
    // batches; the allocation-free call runs neither and creates nothing
    std::lock_guard<std::mutex> lock(g_res_mutex);
    DeviceRes *res = nullptr;
    if (!fixed_scratch && (rc = device_res(device, &res))) return rc;
    CallScratch mem;
    mem.fixed = (char *)fixed;
    mem.cap = fixed_cap;

    // ---- schedule choice per instance
    const size_t budget = (size_t)lds_budget_bytes();
    int n_cu = 256;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    std::vector<char> use_grid(n_inst, 0);
    int64_t r_batch = 0;
    for (int i = 0; i < n_inst; ++i) r_batch += states[i].a.rows;
    for (int i = 0; i < n_inst; ++i) {
        const fsmt_xbdd *h = insts[i];
        const PersistentGeom G = persistent_geom(insts, std::vector<int>{i}, budget);
        const bool fits = G.waves > 0;
        // the instance's schedule: its entry of inst_schedule if set, else the call's
        const int sched = (O.inst_schedule && O.inst_schedule[i] != 0) ? O.inst_schedule[i] : O.schedule;
        if (sched < 0 || sched > 2) return set_error(FSMT_EINVAL, "instance %d: schedule %d unknown", i, sched);
        if (fixed_scratch && sched == 2)
            return set_error(FSMT_EUNSUPPORTED, "the allocation-free call runs the persistent schedule only");
        if ((sched == 1 || fixed_scratch) && !fits)
            return set_error(FSMT_EUNSUPPORTED, "instance %d: restart state (%zu B) does not fit the persistent "
                             "schedule's LDS (%zu B)", i, G.state_f * sizeof(float), budget);
        // big diagrams are evaluated level by level by their own kernel, in the grid schedule
        if ((sched == 1 || fixed_scratch) && h->n_big > 0)
            return set_error(FSMT_EUNSUPPORTED, "instance %d: %d big diagrams need the grid schedule", i, h->n_big);
        use_grid[i] = sched == 2 || !fits || h->n_big > 0 ||
                      (sched == 0 && !fixed_scratch && prefer_grid(h, states[i].a.rows, r_batch, G.waves, n_cu));
    }
    std::vector<int> ia, ib;
    for (int i = 0; i < n_inst; ++i) (use_grid[i] ? ib : ia).push_back(i);
    // the persistent launch takes the largest state and message store of its instances: while
    // that leaves no room for a wave, the instance with the largest state goes to the grid
    // schedule (the persistent schedule only when it was asked for)
    PersistentGeom G;
    while (!ia.empty()) {
        G = persistent_geom(insts, ia, budget);
        if (G.waves > 0) break;
        bool forced = O.schedule == 1 || fixed_scratch;
        for (int i : ia) forced = forced || (O.inst_schedule && O.inst_schedule[i] == 1);
        if (forced)
            return set_error(FSMT_EUNSUPPORTED, "the instances' combined restart state and message store do not fit "
                             "one persistent workgroup's LDS (%zu B)", budget);
        auto big = std::max_element(ia.begin(), ia.end(), [&](int x, int y) {
            return state_floats_of(insts[x]) < state_floats_of(insts[y]);
        });
        ib.push_back(*big);
        ia.erase(big);
    }
    std::sort(ib.begin(), ib.end());

    hipStream_t st = (hipStream_t)stream;
    // the grid part runs on the device's fork stream, concurrently with the persistent launch
    hipStream_t gst = st;
    if (!ia.empty() && !ib.empty()) {
        gst = res->fork;
        if (hipEventRecord(res->ev_fork, st) != hipSuccess || hipStreamWaitEvent(gst, res->ev_fork, 0) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FSMT_EHIP, "stream fork failed");
        }
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
        P.spin_limit = O.spin_limit > 0 ? (uint32_t)O.spin_limit : kSpinLimit;
        for (int t = 0; t < O.n_levels; ++t) P.kappas[t] = O.kappas[t];
        std::vector<InstDesc> desc(ia.size());
        int64_t total_r = 0, min_tasks = INT64_MAX, part_floats = 0;
        for (int i : ia) {
            total_r += states[i].a.rows;
            min_tasks = std::min<int64_t>(min_tasks, insts[i]->n_pos / 64);
        }
        const int msg = G.msg, waves = G.waves;
        const size_t lds = G.lds;
        auto kernel_of = [&](bool cl) -> const void * { return solve_kernel_fn(msg, cl, G.cf); };
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
            // per step and keeps every workgroup resident. Measured per PGD step: placement
            // of 150 rectangles (182 tasks per restart, 8 waves), 16 restarts: 306 us at
            // k = 1, 163 at 2, 89 at 4, 59 at 8; scheduling 200 jobs x 10 machines (66 tasks,
            // 16 waves), 64 restarts: 22.8 us at k = 1, 21.9 at 2, 22.9 at 4.
            const int64_t resd = resident_of(true);
            while (k < 16 && min_tasks >= (int64_t)2 * (2 * k) * waves && total_r * 2 * k <= resd) k *= 2;
        }
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
        P.lds_nodes = G.maxn;
        P.lds_slots = G.maxs;
        P.state_floats = (int32_t)G.state_f;
        P.waves = waves;
        // scratch: descriptors | stop flags [n] | abort flag | barriers [R] | level results [2][2R] | partials [2]
        void *dbuf = nullptr;
        const size_t desc_bytes = sizeof(InstDesc) * desc.size();
        const size_t off_flag = (desc_bytes + 255) / 256 * 256;
        const size_t n_int = desc.size() + 1 + 5 * (size_t)total_r;
        const size_t off_part = off_flag + (n_int * sizeof(int32_t) + 255) / 256 * 256;
        rc = mem.get(off_part + sizeof(float) * (size_t)part_floats, st, &dbuf);
        if (!rc) {
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
            // flags, barriers and level results start at zero (a fill kernel, not a memset:
            // the call may be captured into a graph); the partials are written before read
            if (hipMemcpyAsync(dbuf, desc.data(), desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
                fill_i32(ints, (int64_t)n_int, 0, st) != FSMT_OK) {
                (void)hipGetLastError();
                rc = set_error(FSMT_EHIP, "descriptor upload failed");
            } else {
                const dim3 g((unsigned)wg), b(64 * waves);
                const InstDesc *d = (const InstDesc *)dbuf;
                void *args[] = {(void *)&d, (void *)&P, (void *)&flags, (void *)&abort_flag};
                const hipError_t le = hipLaunchKernel(kernel_of(k > 1), g, b, args, lds, st);
                rc = le != hipSuccess ? set_error(FSMT_EHIP, "solver kernel: %s", hipGetErrorString(le))
                                      : launch_status("solver kernel");
            }
            mem.put(dbuf, st);
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
        const size_t total = off_grd + sizeof(float) * (size_t)scratch_floats;
        void *buf = nullptr;
        if (!rc) rc = mem.get(total, gst, &buf);
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
                (void)hipGetLastError();
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
                plan.cf = 0;
                for (size_t q = 0; q < ib.size(); ++q) plan.cf = std::max(plan.cf, closed_level(insts[ib[q]]));
                // each replay of the level sequence advances every running restart by one
                // level (the kernels read each restart's level from memory and skip finished
                // restarts); levels below level_begin are complete by the caller's word, so
                // they are not replayed
                const int replays = std::max(0, O.n_levels - std::min(O.level_begin, O.n_levels));
                rc = run_grid_schedule((const GridInst *)buf, (int)gi.size(), S, plan, replays, gst, res->cap,
                                       res->retired);
            }
            mem.put(buf, gst);
        }
    }

    if (gst != st) {
        if (hipEventRecord(res->ev_join, gst) != hipSuccess || hipStreamWaitEvent(st, res->ev_join, 0) != hipSuccess) {
            (void)hipGetLastError();
            if (!rc) rc = set_error(FSMT_EHIP, "stream join failed");
        }
    }
    return rc;
}

}  // namespace fsmt

extern "C" fsmt_status fsmt_solve_batched(const fsmt_xbdd *const *insts, int32_t n_inst, const fsmt_solve_opts *opts,
                                          const fsmt_solve_state *states, void *stream) {
    return solve_impl(insts, n_inst, opts, states, stream, nullptr, 0);
}

// ---- allocation-free variant: the call's device memory (descriptors, flags, cluster
// barriers and partial gradients) is carved from this array, one copy per device, held until
// the process ends. In host code the name is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, once per device with that device current.
static __device__ __align__(256) char scratch[FSMT_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mutex;
static void *g_scratch_ptr[kMaxDevices];

extern "C" fsmt_status fsmt_solve_batched_noalloc(const fsmt_xbdd *const *insts, int32_t n_inst,
                                                  const fsmt_solve_opts *opts, const fsmt_solve_state *states,
                                                  void *stream) {
    clear_error();
    if (!insts || n_inst <= 0 || !insts[0]) return set_error(FSMT_EINVAL, "null argument or no instance");
    fsmt_status rc = select_device(insts[0]);
    if (rc) return rc;
    const int device = insts[0]->device;
    if (device < 0 || device >= kMaxDevices) return set_error(FSMT_EINVAL, "device %d out of range", device);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[device]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                return set_error(FSMT_EHIP, "address of the solver scratch on device %d: %s", device,
                                 hipGetErrorString(e));
            }
            g_scratch_ptr[device] = p;
        }
        base = g_scratch_ptr[device];
    }
    return solve_impl(insts, n_inst, opts, states, stream, base, (size_t)FSMT_NOALLOC_SCRATCH_BYTES);
}

extern "C" fsmt_status fsmt_solve_status(const fsmt_solve_state *states, int32_t n_inst, void *stream) {
    clear_error();
    if (!states || n_inst <= 0) return set_error(FSMT_EINVAL, "null argument or no instance");
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        return set_error(FSMT_EHIP, "stream synchronize: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < n_inst; ++i) {
        const int R = states[i].a.rows;
        if (R <= 0 || !states[i].verdict) return set_error(FSMT_EINVAL, "instance %d: no restarts or no verdict", i);
        std::vector<int32_t> v((size_t)R);
        if (hipMemcpy(v.data(), states[i].verdict, sizeof(int32_t) * R, hipMemcpyDeviceToHost) != hipSuccess) {
            const hipError_t e = hipGetLastError();
            return set_error(FSMT_EHIP, "reading verdicts: %s", hipGetErrorString(e));
        }
        for (int r = 0; r < R; ++r)
            if (v[r] == -2)
                return set_error(FSMT_EABORTED, "instance %d, restart %d: a cluster barrier gave up waiting; the "
                                 "state holds its last completed level", i, r);
    }
    return FSMT_OK;
}
