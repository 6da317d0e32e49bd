// Grid schedule of the batched solver, for instances whose restart state does not fit in
// LDS (or whose restarts are too few to fill the device from one workgroup each).
//
// One annealing level is a fixed sequence of grid-wide kernels over all such instances:
//   begin  : per restart, decide whether it runs this level; zero its counters
//   K x  { sweep : forward + reverse sweep of every (constraint, restart) lane of every
//                  instance (waves as in the per-call kernel, lanes of inactive restarts
//                  skip their work), gradient scatter into the instance's gradient arrays
//          step  : per restart (one block), projected step on the box / unit atoms,
//                  gradient map norm, early end of the level once ||g||^2 <= eps^2 }
//   check  : exact check of every (constraint, restart)
//   end    : per restart, ERWA update of its weights, level counter, verdict, stop flag
// Every kernel reads the level of its restart from device memory, so the sequence is
// captured once into a hipGraph and replayed once per level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "eval_task.hpp"
#include "solve_grid.hpp"

namespace fsmt {

__device__ __forceinline__ int find_base32(const GridInst *I, int n, int64_t key, int which) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = which == 0 ? I[mid].task_base
                          : which == 1 ? (int64_t)I[mid].rbase
                          : which == 2 ? I[mid].check_base
                                       : I[mid].level_base;
        if (b <= key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Per restart: does it run this level?
__global__ void grid_begin_kernel(const GridInst *insts, int n_inst, GridShared S) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= S.total_r) return;
    const int ii = find_base32(insts, n_inst, g, 1);
    const GridInst &I = insts[ii];
    const int r = g - I.rbase;
    const bool done = I.verdict[r] == 1 && S.stop_mode != 0;
    const bool stopped = S.stop_mode == 2 && S.stop_flags[ii] != 0;
    const int act = (!done && !stopped && I.level_done[r] < S.n_levels) ? 1 : 0;
    S.active[g] = act;
    S.stepping[g] = act;
    S.obj_acc[g] = 0.0f;
    if (act) {
        I.n_unsat[r] = 0;
        if (I.verdict[r] < 0) I.verdict[r] = 0;   // an earlier call gave up: resume as not SAT
    }
}

// Forward + reverse sweep over every instance's (constraint, restart) lanes.
template <int V, int kCF>
__global__ void __launch_bounds__(256) grid_sweep_kernel(const GridInst *insts, int n_inst, GridShared S) {
    using Ms = typename MsgOf<V>::type;
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, wib = wave_id(), wpb = blockDim.x >> 6;
    const int NN = S.lds_nodes + 2, SS = S.lds_slots;
    FSMT_MSG_STORE(Ms, W, lds + (size_t)wib * (2 * NN + 4 * SS) * 64, NN, SS, lane);
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    // objective partials are carried across this wave's tasks while they stay in one
    // instance (R <= 64: a lane's restart is fixed there) and flushed on a change
    int cur = -1, cur_rpad = 64, cur_rbase = 0, cur_R = 0;
    float oacc = 0.0f;
    auto flush = [&]() {
        if (cur < 0) return;
        for (int off = 32; off >= cur_rpad; off >>= 1) oacc += __shfl_xor(oacc, off, 64);
        if (lane < cur_rpad && lane < cur_R && oacc != 0.0f) atomic_add_f32(S.obj_acc + cur_rbase + lane, oacc);
        oacc = 0.0f;
    };
    for (int64_t task = (int64_t)blockIdx.x * wpb + wib; task < S.total_tasks; task += n_waves) {
        const int ii = find_base32(insts, n_inst, task, 0);
        const GridInst &I = insts[ii];
        const int64_t lt = task - I.task_base;
        int pos, r;
        if (I.R_pad <= 64) {
            pos = (int)(lt * (64 >> I.log2_rpad)) + (lane >> I.log2_rpad);
            r = lane & (I.R_pad - 1);
        } else {
            const int wpc = I.R_pad >> 6;
            pos = (int)(lt / wpc);
            r = (int)(lt % wpc) * 64 + lane;
        }
        if (ii != cur) {
            flush();
            cur = ii;
            cur_rpad = I.R_pad <= 64 ? I.R_pad : 64;
            cur_rbase = I.rbase;
            cur_R = I.R <= 64 ? I.R : 0;
        }
        const bool r_ok = r < I.R && S.stepping[I.rbase + r] != 0;
        const TabView T = I.T;
        const GlobalState st{View{I.a, I.R, T.n_bool, I.a_sr, 1}, View{I.b, I.R, T.n_real, I.b_sr, 1}};
        // gradients restart-contiguous: one wave-wide atomic of a constraint group touches
        // the R_pad consecutive restarts of one variable, one cache line for R_pad <= 16
        const GlobalScatter sc{View{I.ga, I.R, T.n_bool, 1, I.R}, View{I.gb, I.R, T.n_real, 1, I.R},
                               I.R_pad < 64 ? I.R_pad : 64};
        const TaskCtx t = task_ctx(T, pos, r, r_ok);
        if (t.B.big) continue;   // evaluated by grid_level_kernel
        const double kappa = t.valid ? S.kappas[I.level_done[r]] : 0.0;
        const bool hard = isinf(kappa);
        const float wc = t.valid ? I.w[(int64_t)r * T.n_cons + t.c] : 0.0f;   // requested before the forward pass
        const float unsat = task_eval<true, kCF>(T, t, st, kappa, hard, wc, sc, W, lane);
        if (I.R_pad <= 64) {
            oacc += wc * unsat;
        } else if (r < I.R && wc * unsat != 0.0f) {
            atomic_add_f32(S.obj_acc + I.rbase + r, wc * unsat);
        }
    }
    flush();
}

// Big diagrams: one wavefront per (big constraint, chunk of restarts) over every instance,
// level by level (level_eval), into the same gradient rows and objective accumulators.
__global__ void __launch_bounds__(256) grid_level_kernel(const GridInst *insts, int n_inst, GridShared S) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, wib = wave_id(), wpb = blockDim.x >> 6;
    const LevelRows W = LevelRows::at(lds + (size_t)wib * level_wave_floats(S.level_nodes, S.level_slots),
                                      S.level_nodes, S.level_slots);
    WaveObjAcc oa{S.obj_acc};
    // chunk-major task order inside an instance: a wave's consecutive tasks share their
    // restart chunk, so the objective's partial sums stay in lanes
    for (int64_t task = (int64_t)blockIdx.x * wpb + wib; task < S.level_tasks; task += (int64_t)gridDim.x * wpb) {
        const int ii = find_base32(insts, n_inst, task, 3);
        const GridInst &I = insts[ii];
        const int64_t lt = task - I.level_base;
        const int ci = (int)(lt / I.n_big), q = (int)(lt - (int64_t)ci * I.n_big);
        const int r0 = ci * S.level_chunk, r1 = r0 + S.level_chunk < I.R ? r0 + S.level_chunk : I.R;
        oa.begin(I.rbase + r0, r1 - r0, lane);
        const TabView T = I.T;
        const GlobalState st{View{I.a, I.R, T.n_bool, I.a_sr, 1}, View{I.b, I.R, T.n_real, I.b_sr, 1}};
        const GlobalScatter sc{View{I.ga, I.R, T.n_bool, 1, I.R}, View{I.gb, I.R, T.n_real, 1, I.R}, 64};
        const LevelCtx L = level_ctx(T, I.lev, I.big_pos[q]);
        level_stage_nodes(T, L, W, lane);
        for (int r = r0; r < r1; ++r) {
            if (!S.stepping[I.rbase + r]) continue;   // uniform: one restart at a time
            const double kappa = S.kappas[I.level_done[r]];
            const float wc = I.w[(int64_t)r * T.n_cons + L.c];
            const float unsat = level_eval(T, L, st, sc, r, kappa, isinf(kappa), wc, true, W, lane);
            oa.add(r - r0, wc * unsat, lane);
        }
    }
    oa.flush(lane);
}

// Projected step, one block per restart.
__global__ void __launch_bounds__(256) grid_step_kernel(const GridInst *insts, int n_inst, GridShared S) {
    extern __shared__ float sm[];
    const int g = blockIdx.x;
    const int ii = find_base32(insts, n_inst, g, 1);
    const GridInst &I = insts[ii];
    const int r = g - I.rbase;
    if (!S.stepping[g]) return;
    const int n = I.T.n_bool, m = I.T.n_real;
    const gptr<float> arow = I.a + (int64_t)r * I.a_sr, brow = I.b + (int64_t)r * I.b_sr;
    const gptr<float> gacol = I.ga + r, gbcol = I.gb + r;   // element i at i * R
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float x = arow[i], y = x - S.eta_a * gacol[(int64_t)i * I.R];
        const float p = y < -1.0f ? -1.0f : (y > 1.0f ? 1.0f : y);
        arow[i] = p;
        gacol[(int64_t)i * I.R] = 0.0f;
        const float q = (x - p) / S.eta_a;
        acc += q * q;
    }
    if (I.hs.n == 0) {
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            const float x = brow[j], y = x - S.eta_b * gbcol[(int64_t)j * I.R];
            const float p = y < I.T.real_lo[j] ? I.T.real_lo[j] : (y > I.T.real_hi[j] ? I.T.real_hi[j] : y);
            brow[j] = p;
            gbcol[(int64_t)j * I.R] = 0.0f;
            const float q = (x - p) / S.eta_b;
            acc += q * q;
        }
    } else {
        float *y = sm, *pb = sm + m, *ph = sm + 2 * m;
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            y[j] = brow[j] - S.eta_b * gbcol[(int64_t)j * I.R];
            gbcol[(int64_t)j * I.R] = 0.0f;
        }
        project_dykstra(y, pb, ph, I.T.real_lo, I.T.real_hi, m, I.hs);
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            const float x = brow[j], p = y[j];
            brow[j] = p;
            const float q = (x - p) / S.eta_b;
            acc += q * q;
        }
    }
    const float gsq = block_sum(acc);
    if (threadIdx.x == 0) {
        I.obj[r] = S.obj_acc[g];
        S.obj_acc[g] = 0.0f;
        I.steps_done[r] += 1;
        if (gsq <= S.eps2) S.stepping[g] = 0;
    }
}

// Exact check: one 256-thread block per (instance, restart, 256-constraint group).
__global__ void __launch_bounds__(256) grid_check_kernel(const GridInst *insts, int n_inst, GridShared S) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = blockIdx.x;
    const int ii = find_base32(insts, n_inst, blk, 2);
    const GridInst &I = insts[ii];
    const int64_t lb = blk - I.check_base;
    const int groups = (I.T.n_cons + 255) / 256;
    const int r = (int)(lb / groups);
    const int c64 = (int)(lb % groups) * 256 + (threadIdx.x & ~63);
    if (!S.active[I.rbase + r]) return;
    const int c = c64 + lane;
    const int C = I.T.n_cons, nw = (C + 31) >> 5;
    const GlobalState st{View{I.a, I.R, I.T.n_bool, I.a_sr, 1}, View{I.b, I.R, I.T.n_real, I.b_sr, 1}};
    const bool sat = c < C ? walk_state(I.T, st, c, r) : false;
    const uint64_t mask = __ballot(sat);
    const uint64_t valid = __ballot(c < C);
    if (lane == 0 && valid) {
        const gptr<uint32_t> row = I.sat_bits + (int64_t)r * nw;
        row[c64 >> 5] = (uint32_t)mask;
        if ((c64 >> 5) + 1 < nw) row[(c64 >> 5) + 1] = (uint32_t)(mask >> 32);
        atomicAdd((int32_t *)(I.n_unsat + r), (int)__popcll(valid & ~mask));
    }
}

// ERWA, level counter and verdict, one block per restart.
__global__ void __launch_bounds__(1024) grid_end_kernel(const GridInst *insts, int n_inst, GridShared S) {
    const int g = blockIdx.x;
    const int ii = find_base32(insts, n_inst, g, 1);
    const GridInst &I = insts[ii];
    const int r = g - I.rbase;
    if (!S.active[g]) return;
    const int C = I.T.n_cons, nw = (C + 31) >> 5;
    const int level = I.level_done[r];
    const bool update = ((level + 1) % S.tau) == 0;
    const gptr<float> wr = I.w + (int64_t)r * C, hr = I.hist + (int64_t)r * C;
    const gptr<uint32_t> br = I.sat_bits + (int64_t)r * nw;
    float ws = 0.0f;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const float viol = ((br[c >> 5] >> (c & 31)) & 1u) ? 0.0f : 1.0f;
        float h = S.rho * hr[c] + viol, wv = wr[c];
        if (update) {
            wv *= powf(S.gamma, h);
            h = 1.0f;
            wr[c] = wv;
        }
        hr[c] = h;
        ws += wv;
    }
    ws = block_sum(ws);
    if (update && S.normalize) {
        const float scale = (float)C / ws;
        for (int c = threadIdx.x; c < C; c += blockDim.x) wr[c] *= scale;
    }
    if (threadIdx.x == 0) {
        I.level_done[r] = level + 1;
        if (I.n_unsat[r] == 0) {
            I.verdict[r] = 1;
            if (S.stop_mode == 2) atomicExch(S.stop_flags + ii, 1);
        }
    }
}

static fsmt_status launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FSMT_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FSMT_OK;
}

// Enqueue one level's kernel sequence on st.
template <int kCF>
static void launch_sweep(const GridPlan &P, dim3 g, dim3 b, hipStream_t st, const GridInst *d_insts, int n_inst,
                         const GridShared &S) {
    if (P.msg == kMsgSmall)
        hipLaunchKernelGGL((grid_sweep_kernel<kMsgSmall, kCF>), g, b, 0, st, d_insts, n_inst, S);
    else if (P.msg == kMsgMedium)
        hipLaunchKernelGGL((grid_sweep_kernel<kMsgMedium, kCF>), g, b, 0, st, d_insts, n_inst, S);
    else if (P.msg == kMsgLarge)
        hipLaunchKernelGGL((grid_sweep_kernel<kMsgLarge, kCF>), g, b, 0, st, d_insts, n_inst, S);
    else
        hipLaunchKernelGGL((grid_sweep_kernel<kMsgLds, kCF>), g, b, P.sweep_lds, st, d_insts, n_inst, S);
}

static fsmt_status enqueue_level(const GridInst *d_insts, int n_inst, const GridShared &S, const GridPlan &P,
                                 hipStream_t st) {
    fsmt_status rc;
    hipLaunchKernelGGL(grid_begin_kernel, dim3((S.total_r + 255) / 256), dim3(256), 0, st, d_insts, n_inst, S);
    if ((rc = launch_status("grid begin"))) return rc;
    for (int k = 0; k < P.steps; ++k) {
        const dim3 g(P.sweep_blocks), b(64 * P.sweep_wpb);
        if (P.cf == 0)
            launch_sweep<0>(P, g, b, st, d_insts, n_inst, S);
        else if (P.cf == 1)
            launch_sweep<1>(P, g, b, st, d_insts, n_inst, S);
        else if (P.cf == 2)
            launch_sweep<2>(P, g, b, st, d_insts, n_inst, S);
        else
            launch_sweep<3>(P, g, b, st, d_insts, n_inst, S);
        if ((rc = launch_status("grid sweep"))) return rc;
        if (P.level_blocks > 0) {
            hipLaunchKernelGGL(grid_level_kernel, dim3(P.level_blocks), dim3(64 * P.level_wpb), P.level_lds, st, d_insts,
                               n_inst, S);
            if ((rc = launch_status("grid level"))) return rc;
        }
        hipLaunchKernelGGL(grid_step_kernel, dim3(S.total_r), dim3(256), P.step_lds, st, d_insts, n_inst, S);
        if ((rc = launch_status("grid step"))) return rc;
    }
    if (P.check_blocks > 0) {
        hipLaunchKernelGGL(grid_check_kernel, dim3((unsigned)P.check_blocks), dim3(256), 0, st, d_insts, n_inst, S);
        if ((rc = launch_status("grid check"))) return rc;
    }
    hipLaunchKernelGGL(grid_end_kernel, dim3(S.total_r), dim3(1024), 0, st, d_insts, n_inst, S);
    return launch_status("grid end");
}

void reap_retired(std::vector<GraphRetired> &list) {
    size_t keep = 0;
    for (size_t i = 0; i < list.size(); ++i) {
        const hipError_t q = hipEventQuery(list[i].done);
        if (q == hipSuccess) {
            (void)hipGraphExecDestroy(list[i].exec);
            (void)hipGraphDestroy(list[i].graph);
            (void)hipEventDestroy(list[i].done);
        } else {
            (void)hipGetLastError();   // "not ready" is not an error of the next call
            list[keep++] = list[i];
        }
    }
    list.resize(keep);
}

fsmt_status run_grid_schedule(const GridInst *d_insts, int n_inst, const GridShared &S, const GridPlan &P,
                              int n_levels, hipStream_t st, hipStream_t cap, std::vector<GraphRetired> &retired) {
    if (n_levels <= 0 || n_inst == 0) return FSMT_OK;
    // capture one level into a graph on the capture stream, replay it once per level
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = cap != nullptr && P.use_graph && n_levels > 1;
    if (use_graph && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) use_graph = false;
    if (use_graph) {
        fsmt_status rc = enqueue_level(d_insts, n_inst, S, P, cap);
        hipError_t e = hipStreamEndCapture(cap, &graph);
        if (rc || e != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            if (graph) (void)hipGraphDestroy(graph);
            graph = nullptr;
            exec = nullptr;
            use_graph = false;
        }
    }
    fsmt_status rc = FSMT_OK;
    for (int t = 0; t < n_levels && !rc; ++t) {
        if (use_graph) {
            if (hipGraphLaunch(exec, st) != hipSuccess) {
                (void)hipGetLastError();
                rc = set_error(FSMT_EHIP, "hipGraphLaunch failed");
            }
        } else {
            rc = enqueue_level(d_insts, n_inst, S, P, st);
        }
    }
    if (exec) {
        // the executable may be destroyed only after its launches finished: an event after
        // them marks that point, and a later call destroys it
        hipEvent_t done = nullptr;
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess && hipEventRecord(done, st) == hipSuccess) {
            retired.push_back(GraphRetired{exec, graph, done});
        } else {
            (void)hipGetLastError();
            if (done) (void)hipEventDestroy(done);
            (void)hipStreamSynchronize(st);   // no event to wait on: the only safe point is now
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            if (!rc) rc = set_error(FSMT_EHIP, "event creation failed");
        }
    }
    return rc;
}

}  // namespace fsmt
