// Descriptors of the grid schedule of the batched solver (see solve_grid.hip).
#pragma once
#include <vector>

#include "eval_task.hpp"

namespace fsmt {

struct GridInst {
    TabView T;
    HalfSpaces hs;
    gptr<float> a, b, ga, gb;       // row-major [R][n] rows with unit column stride
    int64_t a_sr, b_sr;   // row strides of a, b; ga, gb are restart-contiguous [n][R] work arrays
    gptr<float> w, hist;            // [R][C]
    gptr<uint32_t> sat_bits;
    gptr<int32_t> n_unsat, verdict, level_done, steps_done;
    gptr<float> obj;
    int32_t R, R_pad, log2_rpad, rbase;   // rbase: first global restart index
    int64_t task_base;                    // first sweep task (wave) of this instance
    int64_t check_base;                   // first check block of this instance
    cptr<int32_t> lev, big_pos;           // level starts and positions of big diagrams
    int32_t n_big, pad;
    int64_t level_base;                   // first level-kernel task of this instance
};

struct GridShared {
    const double *kappas;           // device [n_levels]
    int32_t *active, *stepping;     // [total_r]
    float *obj_acc;                 // [total_r]
    int32_t *stop_flags;            // [n_inst]
    int32_t total_r, n_levels, stop_mode, tau, normalize;
    int32_t lds_nodes, lds_slots;
    float eta_a, eta_b, eps2, rho, gamma;
    int64_t total_tasks;
    int64_t level_tasks;            // (big constraint, restart chunk) tasks over all instances
    int32_t level_nodes, level_slots;   // level kernel LDS rows (max over big templates)
    int32_t level_chunk, pad2;      // restarts per level task
};

struct GridPlan {
    int steps;
    int sweep_blocks, sweep_wpb;
    int msg;                        // message-store variant of the sweep (MsgVariant)
    int level_blocks, level_wpb;    // level-synchronous kernel for big diagrams (0 blocks: none)
    size_t level_lds;
    size_t sweep_lds, step_lds;
    int64_t check_blocks;
    bool use_graph;
    int cf;                         // closed-form level of the sweep (largest over the instances)
};

// An instantiated level graph whose replays may still be running: destroyed once the event
// recorded after its last replay has completed (checked without blocking).
struct GraphRetired {
    hipGraphExec_t exec;
    hipGraph_t graph;
    hipEvent_t done;
};
void reap_retired(std::vector<GraphRetired> &list);

// Enqueue n_levels replays of one level's kernel sequence on st (captured into a graph on the
// stream cap). Does not block the host: the graph joins `retired` after its launches.
fsmt_status run_grid_schedule(const GridInst *d_insts, int n_inst, const GridShared &S, const GridPlan &P,
                              int n_levels, hipStream_t st, hipStream_t cap, std::vector<GraphRetired> &retired);

// The batched solver (fsmt_solve_batched). fixed: null to allocate the call's device memory
// stream-ordered, else a device buffer of fixed_cap bytes to carve it from (then only the
// persistent schedule runs, and nothing is allocated).
fsmt_status solve_impl(const fsmt_xbdd *const *insts, int32_t n_inst, const fsmt_solve_opts *opts,
                       const fsmt_solve_state *states, void *stream, void *fixed, size_t fixed_cap);

}  // namespace fsmt
