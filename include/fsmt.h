/*
 * fsmt.h - C ABI of the MI355X (gfx950) FourierSMT hot-path library.
 *
 * The library evaluates the relaxed SMT(LRA) objective of FourierSMT (arXiv 2603.22877)
 * as the circuit-output probability (COP) of each constraint's extended binary decision
 * diagram (xBDD), its gradient by a reverse sweep, a projected-gradient step, and the
 * rounding plus exact satisfaction check, for a batch of R candidate points ("restarts").
 *
 * Conventions (paper, Supplementary Note 1, Cor. "xWFE"; Eq. "rounding"; Eq. "sampling"):
 *  - Truth values: -1 = True, +1 = False. A relaxed Boolean a_i in [-1, 1] is True with
 *    probability p_i = (1 - a_i)/2.
 *  - An atom q.y (op) q0 is True under Gaussian smoothing y' ~ N(b, sigma^2 I) with
 *    probability p = erfc(kappa z / (sqrt(2) |q|)) / 2, z = q.b - q0 written in "<=" form
 *    (">=" and ">" atoms are negated), kappa = 1/sigma in [0, +inf]. kappa = 0 gives
 *    p = 1/2; kappa = +inf gives the exact indicator (and no gradient in b).
 *  - Atoms inside one constraint are treated as independent events (product of their
 *    marginal probabilities), as the message-passing algorithm of Supplementary Note 5
 *    (Alg. "Forward Traversal of XBDDs") does.
 *  - Library objective: U_r = sum_c w_{r,c} * P[c False]  (>= 0, zero exactly at satisfying
 *    vertices). The paper's objective is C_sigma = sum_c w_c E[f_c] = 2 U - sum_c w_c
 *    (Eq. "objective"). Gradients returned are grad U (not -grad C_sigma).
 *
 * Memory: every pointer named in a fsmt_view, and obj / gmap_sq / x / sat_bits / n_unsat /
 * verdict, is DEVICE memory on the handle's device, owned by the caller and only read or
 * written while the stream executes the call. fsmt_problem arrays are HOST memory, read
 * only during xbdd_compile. Calls are asynchronous on the given HIP stream (NULL = the
 * default stream) except xbdd_compile / xbdd_free / xbdd_info, which synchronize.
 *
 * Errors: every call returns an fsmt_status (0 = OK, < 0 = error) and never throws;
 * fsmt_last_error() returns the text of the calling thread's last failure. Shape, stride,
 * null-pointer and device checks happen on the host before anything is launched; on an
 * error nothing is launched and outputs are untouched.
 */
#ifndef FSMT_H
#define FSMT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fsmt_status;
enum {
    FSMT_OK = 0,
    FSMT_EINVAL = -1,       /* invalid argument (shape, stride, pointer, value) */
    FSMT_ENOMEM = -2,       /* host or device allocation failed */
    FSMT_EUNSUPPORTED = -3, /* valid input the library does not handle ("=" atoms, ...) */
    FSMT_ELIMIT = -4,       /* a size limit was exceeded (diagram nodes, support size) */
    FSMT_EHIP = -5,         /* a HIP runtime call failed */
    FSMT_EABORTED = -6      /* a solver call ended early (see fsmt_solve_status) */
};

/* atom comparison operators */
enum { FSMT_LE = 0, FSMT_LT = 1, FSMT_GE = 2, FSMT_GT = 3, FSMT_EQ = 4 };
/* constraint kinds: OR of literals, AND, odd parity, not-all-equal, #true <= k, #true >= k,
 * postfix expression over the literal list */
enum { FSMT_CLAUSE = 0, FSMT_AND = 1, FSMT_XOR = 2, FSMT_NAE = 3, FSMT_CARD_LE = 4,
       FSMT_CARD_GE = 5, FSMT_EXPR = 6 };
/* EXPR connectives (negative ops); an op v >= 0 pushes literal v of the constraint.
 * ITE pops else, then, cond (pushed in the order cond, then, else). */
enum { FSMT_X_AND = -1, FSMT_X_OR = -2, FSMT_X_XOR = -3, FSMT_X_NOT = -4, FSMT_X_ITE = -5,
       FSMT_X_TRUE = -6, FSMT_X_FALSE = -7 };

/* SMT(LRA) formula F = AND_c c (paper, "Satisfiability Modulo Theories"; atoms as in the
 * "Walsh-Fourier Expansions" section). Host arrays, caller-owned, read during compile. */
typedef struct {
    int32_t n_bool, n_real, n_atoms, n_cons;
    const int64_t *atom_ptr;   /* [n_atoms+1] CSR offsets into atom_var / atom_coef */
    const int32_t *atom_var;   /* real-variable ids */
    const double *atom_coef;   /* q_ij */
    const double *atom_rhs;    /* [n_atoms] q_i0 */
    const int8_t *atom_op;     /* [n_atoms] FSMT_LE..FSMT_GT (FSMT_EQ -> FSMT_EUNSUPPORTED) */
    const int32_t *con_kind;   /* [n_cons] */
    const int64_t *con_ptr;    /* [n_cons+1] offsets into con_lit */
    const int32_t *con_lit;    /* literal = 2*id + negated; id < n_bool Boolean, else atom id-n_bool */
    const int32_t *con_param;  /* [n_cons] k of the cardinality kinds (may be NULL) */
    const int64_t *expr_ptr;   /* [n_cons+1] offsets into expr_ops (may be NULL if no EXPR) */
    const int32_t *expr_ops;   /* postfix programs of EXPR constraints */
    const double *real_lo;     /* [n_real] box of b, the feasible set of the projection */
    const double *real_hi;     /* [n_real] */
} fsmt_problem;

#define FSMT_HOST_ONLY (-2)   /* compile_opts.device: keep tables on the host (inspection only) */

/* Feasible set D of the projection (Methods, Def. "Projection", Prop. "qp"). */
enum {
    FSMT_PROJ_UNIT = 0,   /* box plus every unit atomic constraint (a constraint that is one atom
                             literal, no Boolean): single-variable ones tighten the box, the
                             others are half-spaces projected by Dykstra's algorithm (default) */
    FSMT_PROJ_BOX = 1     /* the box [-1,1]^n x [real_lo, real_hi] only */
};

/* Where the diagram passes keep a lane's node messages (Eq. "dp" forward masses and
 * reverse probabilities), and whether recognized diagram families (pair disjunctions,
 * guarded disjunctions: see fsmt_xbdd_stats) run as the same message passing with the
 * graph fixed at compile time. All give the same results; the choice is performance only. */
enum {
    FSMT_MSG_AUTO = 0,    /* closed forms where recognized; registers when the largest other
                             diagram fits a compiled bound, else LDS */
    FSMT_MSG_LDS = 1,     /* closed forms where recognized; the wave's LDS columns for the
                             other diagrams (any size) */
    FSMT_MSG_GENERIC = 2  /* every diagram through the general node-by-node passes (registers
                             when small, else LDS) */
};

typedef struct {
    int32_t device;            /* HIP device that holds the tables (-1 = current device,
                                  FSMT_HOST_ONLY = no upload: only xbdd_info and
                                  xbdd_export_diagram accept such a handle) */
    int32_t max_nodes;         /* reject diagrams with more decision nodes (0 = 1024) */
    int32_t projection;        /* FSMT_PROJ_UNIT or FSMT_PROJ_BOX */
    int32_t messages;          /* FSMT_MSG_AUTO, FSMT_MSG_LDS or FSMT_MSG_GENERIC */
    int32_t reserved[4];
} fsmt_compile_opts;

typedef struct {
    int32_t n_bool, n_real, n_atoms, n_cons;
    int64_t total_nodes;       /* sum over constraints of decision nodes |V_c| */
    int32_t n_templates;       /* distinct diagram shapes */
    int32_t max_nodes;         /* largest |V_c| */
    int32_t max_slots;         /* largest support */
    int32_t n_positions;       /* constraint slots after padding each shape bucket to 64 */
    int64_t table_bytes;       /* device bytes of the compiled tables */
    int64_t atom_nnz;
    int32_t n_box_units;       /* single-variable unit atoms folded into the box */
    int32_t n_halfspaces;      /* multi-variable unit atoms kept as half-spaces of D */
    int32_t n_big;             /* constraints with big diagrams (evaluated level by level,
                                  one wavefront per constraint and restart) */
    int32_t n_hs_colors;       /* colour classes of the half-spaces (members share no variable;
                                  the projection handles a class's members in parallel) */
    int32_t n_pair;            /* constraints of the form OR_i (x_2i XOR x_2i+1) OR atoms, whose
                                  forward and reverse sweeps run in closed form */
    int32_t hs_separable;      /* 1: one colour class and at most 4 distinct variables per
                                  half-space; the projection onto D (Prop. "qp") is then solved
                                  exactly per half-space instead of by Dykstra sweeps */
    int32_t n_gd;              /* constraints that are guarded disjunctions: at most two selector
                                  variables choose, per assignment, a disjunction of literals (a
                                  clause; ITE over clauses); forward and reverse sweeps run in
                                  closed form */
    int32_t n_gd_sep;          /* of those, constraints whose two selectors pick their atoms
                                  independently (a rectangle pair's rotation ITE), so the false
                                  mass is the product of one sum per selector */
} fsmt_xbdd_stats;

/* A strided 2-D float view [rows][cols] of device memory: element (r, v) is at
 * data[r*stride_r + v*stride_v] (strides in elements). stride_r = 0 broadcasts one row
 * (allowed for the weight view only). */
typedef struct {
    float *data;
    int32_t rows, cols;
    int64_t stride_r, stride_v;
} fsmt_view;

typedef struct fsmt_xbdd fsmt_xbdd;   /* opaque compiled instance */

/* Text of the calling thread's last error ("" if none). Valid until the next call. */
const char *fsmt_last_error(void);

/*
 * Compile every constraint into an xBDD (Supplementary Note 3, Def. "xBDD": decision nodes
 * are Booleans or atoms; atoms are treated as propositional variables, no pruning), i.e. a
 * reduced ordered BDD over the constraint's distinct variables (Booleans by id, then atoms
 * by id). Nodes are stored in topological order (Alg. "Forward Traversal of XBDDs" visits
 * them sorted); constraints with the same diagram shape share one node table and are
 * grouped in buckets. Tables are uploaded to the device. *out receives a handle owned by
 * the caller (release with xbdd_free). Errors: FSMT_EINVAL (malformed arrays),
 * FSMT_EUNSUPPORTED ("=" atoms), FSMT_ELIMIT (diagram larger than opts->max_nodes),
 * FSMT_ENOMEM, FSMT_EHIP. opts may be NULL.
 */
fsmt_status xbdd_compile(const fsmt_problem *problem, const fsmt_compile_opts *opts,
                         fsmt_xbdd **out);
void xbdd_free(fsmt_xbdd *handle);                          /* NULL is ignored */
fsmt_status xbdd_info(const fsmt_xbdd *handle, fsmt_xbdd_stats *stats);

/*
 * Copy constraint c's compiled diagram to host memory (inspection and tests).
 * nodes: [3*max_nodes] int32 receiving (slot, hi, lo) per decision node in topological
 * order (root first); child index n_nodes is the True terminal, n_nodes+1 the False one.
 * support: [max_slots] int32 receiving the variable id of each slot (Booleans first, then
 * n_bool + atom id). *root is 0, or the terminal index for a constant constraint.
 * Errors: FSMT_EINVAL (bad c, null pointer), FSMT_ELIMIT (buffers too small).
 */
fsmt_status xbdd_export_diagram(const fsmt_xbdd *handle, int32_t c, int32_t max_nodes, int32_t max_slots,
                                int32_t *n_nodes, int32_t *n_slots, int32_t *n_bslots, int32_t *root,
                                int32_t *nodes, int32_t *support);

/* call flags */
enum {
    FSMT_ACCUMULATE = 1   /* add into obj / grads instead of overwriting them */
};

/*
 * Forward pass (Alg. "Forward Traversal of XBDDs"; Supplementary Note 5, Lemma "forward"):
 * literal probabilities from a [R][n_bool] and b [R][n_real] (Eq. "rounding", "sampling"),
 * top-down path masses m_td, and per constraint P[c False] = mass reaching the false
 * terminal. obj[r] = U_r = sum_c w[r][c] P[c False] ([R] device floats, required).
 * w: [R][n_cons] or broadcast [1][n_cons] (stride_r = 0). unsat: optional [R][n_cons]
 * output of P[c False] (data = NULL to skip). kappa = 1/sigma in [0, +inf].
 */
fsmt_status cop_forward(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, double kappa, fsmt_view w,
                        float *obj, fsmt_view unsat, int32_t flags, void *stream);

/*
 * Forward + reverse sweep (Alg. "Backward Traversal of XBDD"; Supplementary Note 5, Lemma
 * "backward", Thm. "Differentiation"): bottom-up masses m_bu(v) = P[reach False from v],
 * dU/dp_v = w_c * sum_{nodes of v} m_td * (m_bu[true child] - m_bu[false child]), then the
 * chain rule dp/da = -1/2 and dp/db_j = -kappa q_j exp(-u^2) / (sqrt(2 pi) |q|)
 * (Supplementary Note 6). grad_a [R][n_bool], grad_b [R][n_real] receive grad U; obj
 * (optional, NULL to skip) receives U. Without FSMT_ACCUMULATE the outputs are zeroed
 * first. Gradient sums use float atomics, so the last bits vary between runs. On instances
 * of at least 8 x 64 constraints per compute unit the call takes stream-ordered work memory
 * (hipMallocAsync / hipFreeAsync on `stream`: per-workgroup gradient rows for up to 16
 * restarts on diagrams of the register message store, else a restart-contiguous gradient
 * stage for 4-64 restarts in gradients that are not restart-contiguous already);
 * FSMT_ENOMEM if that fails.
 */
fsmt_status cop_backward(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, double kappa,
                         fsmt_view w, float *obj, fsmt_view grad_a, fsmt_view grad_b,
                         int32_t flags, void *stream);

/*
 * Projected gradient step (Methods, Eq. "pg1"/"pg2", Def. "Projection", Prop. "qp"), in
 * place on a and b: a <- clamp(a - eta_a grad_a, -1, 1) (the Euclidean projection onto a
 * box is the coordinate-wise clamp) and b <- proj_D(b - eta_b grad_b), where D is the box
 * [real_lo, real_hi] tightened by single-variable unit atoms, intersected with the
 * half-spaces q.b <= q0 - delta of multi-variable unit atoms (delta = 1e-6 (|q0| +
 * sum_j |q_j| max(|lo_j|, |hi_j|)) keeps the rounded point on the satisfied side). The
 * intersection is projected by Dykstra's alternating projections (at most 256 sweeps, until
 * a sweep moves no coordinate by more than 4e-7 (1 + |b|)); when no two half-spaces
 * share a variable and each has at most 4 distinct variables, the projection separates
 * into one closed-form projection per half-space instead (exact up to rounding);
 * and gmap_sq[r] = ||g||^2 of the gradient map g = ((a-a+)/eta_a, (b-b+)/eta_b)
 * (Eq. "grad_map", "critical"); gmap_sq may be NULL. grad_a / grad_b are zeroed after use
 * (so the next cop_backward can run with FSMT_ACCUMULATE). NaN inputs stay NaN.
 */
fsmt_status pgd_step(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, fsmt_view grad_a,
                     fsmt_view grad_b, float eta_a, float eta_b, float *gmap_sq, int32_t flags,
                     void *stream);

/*
 * Rounding and exact check (Alg. "FourierSMT", last lines; Thm. "Soundness"):
 * x_i = True (-1) iff a_i < 0 (so +-0 and NaN round to False); y = b. Atoms are decided
 * exactly: z = sum_j q_j y_j - q0 in FP64 from the float32 y, multiply then add in the
 * input's coefficient order (no fused multiply-add), True iff z <= 0 (z < 0 for strict
 * atoms); NaN compares false. Each diagram is walked from its root.
 * Outputs ([R] leading dimension, contiguous, device):
 *   x [R][n_bool] int8 (+-1; NULL to skip), sat_bits [R][ceil(n_cons/32)] (bit c%32 of word
 *   c/32 set iff constraint c is satisfied), n_unsat [R], verdict [R] (1 = SAT, 0 = UNKNOWN).
 */
fsmt_status round_and_check(const fsmt_xbdd *h, fsmt_view a, fsmt_view b, int8_t *x,
                            uint32_t *sat_bits, int32_t *n_unsat, int32_t *verdict,
                            void *stream);

/*
 * ERWA weight update of Alg. "CLS with Annealing" for level t = level (1-based) from the
 * satisfied-constraint bits of round_and_check: for every constraint
 * h = rho h + [c violated]; if t mod tau == 0: w *= gamma^h and h = 1; then, if normalize,
 * w *= n_cons / sum(w) (keeps the weights finite; the minimizer is scale-invariant).
 * sat_bits [R][ceil(n_cons/32)], w and hist [R][n_cons]: contiguous device arrays.
 */
fsmt_status erwa_update(const fsmt_xbdd *h, int32_t R, const uint32_t *sat_bits, float *w, float *hist,
                        int32_t level, float rho, float gamma, int32_t tau, int32_t normalize,
                        void *stream);

/* ------------------------------------------------------------------ batched solver */

/* Options of the annealed solver (Alg. "CLS with Annealing" around Alg. "FourierSMT"). */
typedef struct {
    const double *kappas;     /* host [n_levels] annealing schedule kappa_t = 1/sigma_t */
    int32_t n_levels;
    int32_t steps_per_level;  /* PGD iterations per level (cap) */
    float eta_a, eta_b;       /* step sizes on U */
    float eps;                /* stop a level early when ||g||^2 <= eps^2 (eps <= 0: never) */
    float rho, gamma;         /* ERWA decay and scaling base */
    int32_t tau;              /* ERWA update period in levels */
    int32_t normalize;        /* renormalize weights to sum n_cons after each update */
    int32_t stop_on_sat;      /* 0 = keep iterating (fixed work, benchmarks); 1 = a restart stops
                                 once its check passes; 2 = additionally every restart of the
                                 same instance stops at its next level boundary */
    int32_t schedule;         /* 0 = automatic, 1 = persistent, 2 = grid (see fsmt_solve_batched) */
    int32_t cluster;          /* persistent schedule: workgroups per restart (0 = automatic) */
    int32_t level_begin;      /* grid schedule: levels below this are complete for every restart
                                 of the call (the caller's word); each restart then runs at most
                                 n_levels - level_begin levels in this call (0: no promise) */
    int32_t spin_limit;       /* polls of a cluster barrier before it gives up (0 = 2^22); a small
                                 value makes an incomplete cluster end the call early */
    const int32_t *inst_schedule; /* host [n_inst] or NULL: per instance 0 = as `schedule`, 1 =
                                 persistent, 2 = grid (a plan chosen by measurement, see the
                                 package's autotuner) */
} fsmt_solve_opts;

/* Per-instance solver state, device memory owned by the caller ([R] rows each). The
 * counters level_done / steps_done and verdict are read at entry (a call resumes where the
 * previous one stopped) and written at exit. */
typedef struct {
    fsmt_view a, b;           /* [R][n_bool], [R][n_real] in/out (row stride >= cols, unit column stride) */
    float *w;                 /* [R][n_cons] in/out weights */
    float *hist;              /* [R][n_cons] in/out ERWA history h */
    float *grad_a, *grad_b;   /* grid schedule work arrays, [n_bool][R], [n_real][R] (may be NULL) */
    uint32_t *sat_bits;       /* [R][ceil(n_cons/32)] out: last check */
    int32_t *n_unsat;         /* [R] out */
    int32_t *verdict;         /* [R] out: 1 = SAT found (state a, b holds the assignment) */
    int32_t *level_done;      /* [R] out: levels completed */
    int32_t *steps_done;      /* [R] out: PGD steps executed */
    float *obj;               /* [R] out: U after the last step */
} fsmt_solve_state;

/*
 * Run the annealed PGD solver for n_inst instances at once, each with its own R restarts
 * (Alg. "CLS with Annealing" around the PGD loop of Alg. "FourierSMT"), fusing forward,
 * reverse sweep, projection, check and ERWA on the device. For every restart and every level
 * t from level_done[r] to n_levels-1 with kappa_t = kappas[t]: projected gradient steps while
 * the gradient map of the last step has ||g||^2 > eps^2 (each restart on its own; at least
 * one and at most steps_per_level steps), then rounding + exact check and the ERWA update
 * (h = rho h + [violated]; every tau levels w *= gamma^h, h = 1, then optional
 * renormalization of w to sum n_cons). A restart whose check reports no violated constraint
 * is SAT (Thm. "Soundness"). At the end of every level a restart's a, b, level_done,
 * steps_done, n_unsat, obj and verdict are written together.
 *
 * Schedules (opts->schedule; 0 picks one per instance from a cost model): persistent, one
 * workgroup (or a cluster of `cluster` co-resident workgroups) per restart with the state
 * in LDS, one launch; grid, one captured graph of grid-wide kernels replayed per level, for
 * states that do not fit in LDS, big diagrams, or too few restarts to fill the device. A
 * batch may mix both (they run concurrently). The grid schedule uses grad_a / grad_b of the
 * state as work arrays when given (else its own): restart-contiguous, grad_a[i * R + r] and
 * grad_b[j * R + r], zero at entry and left zero.
 *
 * Asynchronous on the stream: the call enqueues work and returns without waiting for the
 * device. A cluster whose workgroups were not all resident gives up at a bounded barrier
 * wait (spin_limit): every restart of that launch that was still running then ends with
 * verdict = -2 and the state of its last completed level; fsmt_solve_status reports it.
 * Errors (before anything is launched): FSMT_EINVAL for bad shapes or options, FSMT_ELIMIT
 * for more than 128 levels or diagrams beyond the LDS bounds, FSMT_EUNSUPPORTED when the
 * persistent schedule is asked for but a state does not fit in LDS, an instance has big
 * diagrams, or a forced cluster size cannot be co-resident.
 */
fsmt_status fsmt_solve_batched(const fsmt_xbdd *const *insts, int32_t n_inst,
                               const fsmt_solve_opts *opts, const fsmt_solve_state *states,
                               void *stream);

/*
 * Allocation-free variant of fsmt_solve_batched, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. Same arguments, semantics and results as fsmt_solve_batched restricted to the
 * persistent schedule (schedule 0 or 1; schedule 2 returns FSMT_EUNSUPPORTED, and so does
 * an instance that the persistent schedule cannot take: state beyond LDS, big diagrams).
 * The call's device memory (descriptors, stop and abort flags, cluster barriers, level
 * results and partial gradients) is carved from a library-owned device array of
 * FSMT_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; a call that needs more
 * returns FSMT_ELIMIT before launching anything. The call allocates nothing (no hipMalloc,
 * no stream-ordered allocation, no streams or events); what must start at zero is cleared
 * by a fill kernel on the stream. Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (two streams, or two host threads) race and must be serialized
 * by the caller; calls in order on one stream are safe.
 */
#define FSMT_NOALLOC_SCRATCH_BYTES (8u << 20)
fsmt_status fsmt_solve_batched_noalloc(const fsmt_xbdd *const *insts, int32_t n_inst,
                                       const fsmt_solve_opts *opts, const fsmt_solve_state *states,
                                       void *stream);

/*
 * Outcome of the solver calls enqueued on the stream: synchronizes the stream, then reads
 * every restart's verdict. Returns FSMT_EABORTED (with the instance and restart in
 * fsmt_last_error) if a restart ended with verdict -2, i.e. a call gave up early; the
 * state then holds that restart's last completed level and a new call resumes from there.
 * FSMT_OK otherwise. FSMT_EHIP if the device reported an error.
 */
fsmt_status fsmt_solve_status(const fsmt_solve_state *states, int32_t n_inst, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FSMT_H */
