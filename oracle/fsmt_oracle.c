/*
 * FP64 reference oracle for the FourierSMT hot path.
 *
 * TEST INFRASTRUCTURE ONLY. This file is compiled and called by the test-suite, by the
 * CPU-baseline leg of the benchmark and by the smoke check; the library never links,
 * loads or calls it. It shares no code with the HIP path: it never builds a decision
 * diagram. Every quantity is computed from the original formula of each constraint.
 *
 * What it computes (paper references by section / equation / algorithm):
 *  - Literal probabilities: P[x_i = True] = (1 - a_i)/2 (Eq. "rounding"); for an atom
 *    q.y <= q0 under Gaussian smoothing y ~ N(b, sigma^2 I), P[atom True] =
 *    (1 - d)/2 with d = erf((q.b - q0)/(sqrt(2) sigma |q|)) (Eq. "sampling"),
 *    evaluated as erfc(u)/2 with kappa = 1/sigma.
 *  - Circuit-output probability of each constraint (Supplementary Note 4, Remark COP and
 *    Cor. cop=wfe): the probability mass of the satisfying (P_true) and of the falsifying
 *    (P_false) assignments of the constraint's variables, literals independent. It is
 *    computed by the Shannon expansion f = p f|v=T + (1-p) f|v=F (law of total
 *    probability), stopping as soon as a three-valued evaluation of the original formula
 *    is decided, by plain enumeration of all assignments, or, for large symmetric
 *    constraints with distinct variables, from the distribution of the number of true
 *    literals (Poisson-binomial).
 *  - Gradient: P_false is multilinear in the literal probabilities, so its partial
 *    derivative in p_v is P_false|v=T - P_false|v=F exactly (Supplementary Note 5,
 *    Thm. "Differentiation"); chain rule dp/da = -1/2 and
 *    dp/db_j = -kappa s q_j exp(-u^2) / (sqrt(2 pi) |q|) (Supplementary Note 6, Prop.
 *    "Lipschitz", derivative of d_i).
 *  - Objective U = sum_c w_c P_false,c; the paper's C_sigma = 2U - sum w (Eq. "objective").
 *  - Projected gradient step onto the box (Eq. "pg1"/"pg2", Def. "Projection") and the
 *    gradient map (Eq. "grad_map").
 *  - Rounding x = sgn(a) and the exact check F_w(x, y) = -sum w (Alg. "FourierSMT",
 *    Thm. "Soundness"): the original formula is evaluated with exact FP64 atom tests.
 *  - ERWA weight update of Alg. "CLS with Annealing".
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no FMA contraction, so
 * atom tests are a multiply then an add, each rounded).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* input format (see workloads/format.py) */
enum { O_LE = 0, O_LT = 1, O_GE = 2, O_GT = 3, O_EQ = 4 };
enum { K_CLAUSE = 0, K_AND = 1, K_XOR = 2, K_NAE = 3, K_CARD_LE = 4, K_CARD_GE = 5, K_EXPR = 6 };
enum { E_AND = -1, E_OR = -2, E_XOR = -3, E_NOT = -4, E_ITE = -5, E_TRUE = -6, E_FALSE = -7 };

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EUNSUPPORTED = -3, ORC_ELIMIT = -4 };

typedef struct {
    int32_t n_bool, n_real, n_atoms, n_cons;
    const int64_t *atom_ptr;
    const int32_t *atom_var;
    const double *atom_coef;
    const double *atom_rhs;
    const int8_t *atom_op;
    const int32_t *con_kind;
    const int64_t *con_ptr;
    const int32_t *con_lit;
    const int32_t *con_param;
    const int64_t *expr_ptr;
    const int32_t *expr_ops;
} oproblem;

#define MAX_SUPPORT 64   /* distinct variables per constraint */
#define MAX_LITS 256     /* literal occurrences per constraint */
#define MAX_SHANNON 24   /* largest support expanded by recursion */
#define MAX_STACK 512    /* EXPR evaluation stack */

/* ---------------------------------------------------------------- atoms */

/* z = sum_j q_j y_j - q0, stored order, multiply then add (no contraction) */
static double atom_z(const oproblem *P, int k, const float *y)
{
    double acc = 0.0;
    for (int64_t e = P->atom_ptr[k]; e < P->atom_ptr[k + 1]; ++e) {
        double prod = P->atom_coef[e] * (double)y[P->atom_var[e]];
        acc = acc + prod;
    }
    return acc - P->atom_rhs[k];
}

/* exact truth of atom k at y; NaN compares false */
static int atom_true_at(const oproblem *P, int k, const float *y)
{
    double z = atom_z(P, k, y);
    switch (P->atom_op[k]) {
    case O_LE: return z <= 0.0;
    case O_LT: return z < 0.0;
    case O_GE: return z >= 0.0;
    case O_GT: return z > 0.0;
    default: return z == 0.0;
    }
}

static double atom_norm(const oproblem *P, int k)
{
    double s = 0.0;
    for (int64_t e = P->atom_ptr[k]; e < P->atom_ptr[k + 1]; ++e)
        s += P->atom_coef[e] * P->atom_coef[e];
    return sqrt(s);
}

/* P[atom k True] under y' ~ N(b, I/kappa^2), and dP/dz (z = q.b - q0) */
static double atom_prob(const oproblem *P, int k, const float *b, double kappa, double *dpdz)
{
    double z = atom_z(P, k, b);
    int op = P->atom_op[k];
    if (isinf(kappa)) {           /* sigma = 0: the exact indicator, no gradient */
        *dpdz = 0.0;
        return atom_true_at(P, k, b) ? 1.0 : 0.0;
    }
    double s = (op == O_GE || op == O_GT) ? -1.0 : 1.0;   /* >= flips the side */
    double qn = atom_norm(P, k);
    double u = kappa * s * z / (sqrt(2.0) * qn);
    *dpdz = -kappa * s * exp(-u * u) / (sqrt(2.0 * M_PI) * qn);
    return 0.5 * erfc(u);
}

/* ---------------------------------------------------------- constraint view */

typedef struct {
    int kind, param;
    int n_lits;
    int k;                          /* support size */
    int32_t ids[MAX_SUPPORT];       /* distinct variable ids, ascending */
    int slot[MAX_LITS];             /* literal position -> support slot */
    int neg[MAX_LITS];
    const int32_t *ops;
    int n_ops;
    double p[MAX_SUPPORT];          /* P[variable True] */
    signed char val[MAX_SUPPORT];   /* -1 unassigned, 0 False, 1 True */
} cview;

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static int make_view(const oproblem *P, int c, cview *V)
{
    int64_t l0 = P->con_ptr[c], l1 = P->con_ptr[c + 1];
    V->kind = P->con_kind[c];
    V->param = P->con_param[c];
    V->n_lits = (int)(l1 - l0);
    if (V->n_lits > MAX_LITS) return ORC_ELIMIT;
    int32_t tmp[MAX_LITS];
    for (int t = 0; t < V->n_lits; ++t) tmp[t] = P->con_lit[l0 + t] >> 1;
    qsort(tmp, V->n_lits, sizeof(int32_t), cmp_i32);
    V->k = 0;
    for (int t = 0; t < V->n_lits; ++t)
        if (V->k == 0 || V->ids[V->k - 1] != tmp[t]) {
            if (V->k == MAX_SUPPORT) return ORC_ELIMIT;
            V->ids[V->k++] = tmp[t];
        }
    for (int t = 0; t < V->n_lits; ++t) {
        int32_t id = P->con_lit[l0 + t] >> 1;
        V->neg[t] = P->con_lit[l0 + t] & 1;
        int s = 0;
        while (V->ids[s] != id) ++s;
        V->slot[t] = s;
    }
    V->ops = P->expr_ops + P->expr_ptr[c];
    V->n_ops = (int)(P->expr_ptr[c + 1] - P->expr_ptr[c]);
    for (int s = 0; s < V->k; ++s) V->val[s] = -1;
    return ORC_OK;
}

static int lit_val(const cview *V, int t)
{
    int v = V->val[V->slot[t]];
    return v < 0 ? -1 : (v ^ V->neg[t]);
}

/* three-valued (Kleene) evaluation of the original formula: 1 True, 0 False, -1 undecided */
static int eval3(const cview *V)
{
    int nt = 0, nf = 0, nu = 0;
    if (V->kind != K_EXPR) {
        for (int t = 0; t < V->n_lits; ++t) {
            int v = lit_val(V, t);
            if (v < 0) ++nu; else if (v) ++nt; else ++nf;
        }
    }
    switch (V->kind) {
    case K_CLAUSE: return nt > 0 ? 1 : (nu > 0 ? -1 : 0);
    case K_AND:    return nf > 0 ? 0 : (nu > 0 ? -1 : 1);
    case K_XOR:    return nu > 0 ? -1 : (nt & 1);
    case K_NAE:    return (nt > 0 && nf > 0) ? 1 : (nu > 0 ? -1 : 0);
    case K_CARD_LE:
        if (nt > V->param) return 0;
        if (nt + nu <= V->param) return 1;
        return -1;
    case K_CARD_GE:
        if (nt >= V->param) return 1;
        if (nt + nu < V->param) return 0;
        return -1;
    case K_EXPR: {
        signed char st[MAX_STACK];
        int sp = 0;
        for (int i = 0; i < V->n_ops; ++i) {
            int op = V->ops[i];
            if (op >= 0) { st[sp++] = (signed char)lit_val(V, op); continue; }
            if (op == E_TRUE) { st[sp++] = 1; continue; }
            if (op == E_FALSE) { st[sp++] = 0; continue; }
            if (op == E_NOT) { int x = st[sp - 1]; st[sp - 1] = (signed char)(x < 0 ? -1 : 1 - x); continue; }
            if (op == E_ITE) {
                int e = st[--sp], th = st[--sp], cnd = st[--sp];
                int r = cnd == 1 ? th : cnd == 0 ? e : (th == e && th >= 0 ? th : -1);
                st[sp++] = (signed char)r;
                continue;
            }
            int y = st[--sp], x = st[--sp], r;
            if (op == E_AND) r = (x == 0 || y == 0) ? 0 : (x == 1 && y == 1) ? 1 : -1;
            else if (op == E_OR) r = (x == 1 || y == 1) ? 1 : (x == 0 && y == 0) ? 0 : -1;
            else r = (x < 0 || y < 0) ? -1 : (x ^ y);
            st[sp++] = (signed char)r;
        }
        return st[0];
    }
    }
    return -1;
}

static int validate_expr(const cview *V)
{
    if (V->kind != K_EXPR) return V->kind >= 0 && V->kind <= K_CARD_GE ? ORC_OK : ORC_EINVAL;
    int sp = 0;
    for (int i = 0; i < V->n_ops; ++i) {
        int op = V->ops[i];
        if (op >= 0) { if (op >= V->n_lits) return ORC_EINVAL; ++sp; }
        else if (op == E_TRUE || op == E_FALSE) ++sp;
        else if (op == E_NOT) { if (sp < 1) return ORC_EINVAL; }
        else if (op == E_ITE) { if (sp < 3) return ORC_EINVAL; sp -= 2; }
        else if (op == E_AND || op == E_OR || op == E_XOR) { if (sp < 2) return ORC_EINVAL; --sp; }
        else return ORC_EINVAL;
        if (sp > MAX_STACK) return ORC_ELIMIT;
    }
    return sp == 1 ? ORC_OK : ORC_EINVAL;
}

/* ------------------------------------------------- Shannon expansion with gradients */

/* Returns P_true, P_false of the formula given the assignment of slots < depth, and the
 * derivatives of P_false in p[s] for s >= depth (dF has k entries). */
static void shannon(cview *V, int depth, double *PT, double *PF, double *dF)
{
    int v = eval3(V);
    for (int s = depth; s < V->k; ++s) dF[s] = 0.0;
    if (v >= 0) {
        *PT = v ? 1.0 : 0.0;
        *PF = v ? 0.0 : 1.0;
        return;
    }
    double AT, AF, BT, BF;
    double dAF[MAX_SHANNON], dBF[MAX_SHANNON];
    V->val[depth] = 1;
    shannon(V, depth + 1, &AT, &AF, dAF);
    V->val[depth] = 0;
    shannon(V, depth + 1, &BT, &BF, dBF);
    V->val[depth] = -1;
    double p = V->p[depth];
    *PT = p * AT + (1.0 - p) * BT;
    *PF = p * AF + (1.0 - p) * BF;
    dF[depth] = AF - BF;
    for (int s = depth + 1; s < V->k; ++s)
        dF[s] = p * dAF[s] + (1.0 - p) * dBF[s];
}

/* Count-distribution evaluation for symmetric kinds whose literals use distinct variables. */
static int symmetric_value(int kind, int param, int L, int t)
{
    switch (kind) {
    case K_CLAUSE: return t >= 1;
    case K_AND: return t == L;
    case K_XOR: return t & 1;
    case K_NAE: return t > 0 && t < L;
    case K_CARD_LE: return t <= param;
    case K_CARD_GE: return t >= param;
    }
    return 0;
}

static void count_dist(const double *pi, int L, int skip, double *dist)
{
    dist[0] = 1.0;
    int len = 0;
    for (int l = 0; l < L; ++l) {
        if (l == skip) continue;
        dist[len + 1] = 0.0;
        for (int t = len + 1; t >= 1; --t) dist[t] = dist[t] * (1.0 - pi[l]) + dist[t - 1] * pi[l];
        dist[0] *= (1.0 - pi[l]);
        ++len;
    }
}

static void symmetric_eval(const cview *V, double *PT, double *PF, double *dF)
{
    int L = V->n_lits;
    double pi[MAX_LITS], dist[MAX_LITS + 2];
    for (int t = 0; t < L; ++t) {
        double p = V->p[V->slot[t]];
        pi[t] = V->neg[t] ? 1.0 - p : p;
    }
    count_dist(pi, L, -1, dist);
    double st = 0.0, sf = 0.0;
    for (int t = 0; t <= L; ++t) {
        if (symmetric_value(V->kind, V->param, L, t)) st += dist[t]; else sf += dist[t];
    }
    *PT = st;
    *PF = sf;
    for (int s = 0; s < V->k; ++s) dF[s] = 0.0;
    for (int l = 0; l < L; ++l) {
        count_dist(pi, L, l, dist);   /* distribution of the other L-1 literals */
        double gf = 0.0;              /* d P_false / d pi_l */
        for (int t = 0; t <= L - 1; ++t) {
            int with = symmetric_value(V->kind, V->param, L, t + 1);
            int without = symmetric_value(V->kind, V->param, L, t);
            gf += dist[t] * ((double)(!with) - (double)(!without));
        }
        dF[V->slot[l]] += (V->neg[l] ? -1.0 : 1.0) * gf;
    }
}

static int constraint_cop(cview *V, double *PT, double *PF, double *dF)
{
    int rc = validate_expr(V);
    if (rc) return rc;
    if (V->k <= 12 || (V->k <= MAX_SHANNON && (V->kind == K_EXPR || V->k != V->n_lits))) {
        shannon(V, 0, PT, PF, dF);
        return ORC_OK;
    }
    if (V->kind != K_EXPR && V->k == V->n_lits) {
        symmetric_eval(V, PT, PF, dF);
        return ORC_OK;
    }
    return ORC_ELIMIT;
}

/* ---------------------------------------------------------------- exports */

/* Plain enumeration of the constraint's 2^k assignments (k <= 20), for pinning. */
int oracle_cop_enum(const oproblem *P, int c, const double *pvar /* P[var True] by id */,
                    double *PT, double *PF)
{
    cview V;
    int rc = make_view(P, c, &V);
    if (rc) return rc;
    if ((rc = validate_expr(&V))) return rc;
    if (V.k > 20) return ORC_ELIMIT;
    double st = 0.0, sf = 0.0;
    for (uint32_t m = 0; m < (1u << V.k); ++m) {
        double pr = 1.0;
        for (int s = 0; s < V.k; ++s) {
            V.val[s] = (signed char)((m >> s) & 1);
            double p = pvar[V.ids[s]];
            pr *= V.val[s] ? p : 1.0 - p;
        }
        if (eval3(&V)) st += pr; else sf += pr;
    }
    *PT = st;
    *PF = sf;
    return ORC_OK;
}

/* One constraint at given variable probabilities: P_true, P_false and dP_false/dp by slot
 * order of the sorted distinct variable ids (written to ids_out, size returned in *k). */
int oracle_cop_one(const oproblem *P, int c, const double *pvar, double *PT, double *PF,
                   double *dF_out, int32_t *ids_out, int *k_out)
{
    cview V;
    int rc = make_view(P, c, &V);
    if (rc) return rc;
    for (int s = 0; s < V.k; ++s) V.p[s] = pvar[V.ids[s]];
    double dF[MAX_SUPPORT];
    rc = constraint_cop(&V, PT, PF, dF);
    if (rc) return rc;
    for (int s = 0; s < V.k; ++s) { dF_out[s] = dF[s]; ids_out[s] = V.ids[s]; }
    *k_out = V.k;
    return ORC_OK;
}

/* Evaluate the formula of constraint c at a full truth assignment (val by var id, 0/1). */
int oracle_eval_formula(const oproblem *P, int c, const int8_t *truth)
{
    cview V;
    if (make_view(P, c, &V)) return -1;
    for (int s = 0; s < V.k; ++s) V.val[s] = (signed char)(truth[V.ids[s]] ? 1 : 0);
    return eval3(&V);
}

/* Atom probabilities at one point: p[k], dp/dz[k], z[k] for every atom. */
int oracle_atom_probs(const oproblem *P, const float *b, double kappa, double *p, double *dpdz,
                      double *z)
{
    for (int k = 0; k < P->n_atoms; ++k) {
        if (P->atom_op[k] == O_EQ || P->atom_op[k] < 0 || P->atom_op[k] > O_EQ) return ORC_EUNSUPPORTED;
        p[k] = atom_prob(P, k, b, kappa, &dpdz[k]);
        if (z) z[k] = atom_z(P, k, b);
    }
    return ORC_OK;
}

/*
 * Objective, per-constraint masses and gradient for R points.
 *   a [R][n_bool], b [R][n_real] (float32, as the library receives them)
 *   w [R][C] constraint weights or NULL (all ones)
 *   U [R]; unsat / sat [R][C] or NULL; grad_a [R][n], grad_b [R][m] or NULL;
 *   absg_a, absg_b: sum over constraints of |contribution| per coordinate (or NULL);
 *   sel: subset of constraints (n_sel entries) or NULL for all.
 */
int oracle_objective(const oproblem *P, int R, const float *a, const float *b, double kappa,
                     const double *w, double *U, double *unsat, double *sat, double *grad_a,
                     double *grad_b, double *absg_a, double *absg_b, const int32_t *sel, int n_sel)
{
    int n = P->n_bool, m = P->n_real, C = P->n_cons;
    if (kappa < 0.0 || isnan(kappa)) return ORC_EINVAL;
    int nc = sel ? n_sel : C;
    double *pv = (double *)malloc(sizeof(double) * (size_t)(n + P->n_atoms));
    double *dz = (double *)malloc(sizeof(double) * (size_t)(P->n_atoms + 1));
    if (!pv || !dz) { free(pv); free(dz); return -2; }
    int rc = ORC_OK;
    for (int r = 0; r < R && rc == ORC_OK; ++r) {
        const float *ar = a + (size_t)r * n, *br = b + (size_t)r * m;
        for (int i = 0; i < n; ++i) pv[i] = (1.0 - (double)ar[i]) / 2.0;
        if (!sel) {
            for (int k = 0; k < P->n_atoms; ++k) {
                if (P->atom_op[k] == O_EQ) { rc = ORC_EUNSUPPORTED; break; }
                pv[n + k] = atom_prob(P, k, br, kappa, &dz[k]);
            }
        } else {   /* only the atoms of the selected constraints */
            for (int ci = 0; ci < nc && !rc; ++ci) {
                int c = sel[ci];
                if (c < 0 || c >= C) { rc = ORC_EINVAL; break; }
                for (int64_t l = P->con_ptr[c]; l < P->con_ptr[c + 1]; ++l) {
                    int id = P->con_lit[l] >> 1;
                    if (id < n) continue;
                    int k = id - n;
                    if (P->atom_op[k] == O_EQ) { rc = ORC_EUNSUPPORTED; break; }
                    pv[id] = atom_prob(P, k, br, kappa, &dz[k]);
                }
            }
        }
        if (rc) break;
        if (grad_a) memset(grad_a + (size_t)r * n, 0, sizeof(double) * n);
        if (grad_b) memset(grad_b + (size_t)r * m, 0, sizeof(double) * m);
        if (absg_a) memset(absg_a + (size_t)r * n, 0, sizeof(double) * n);
        if (absg_b) memset(absg_b + (size_t)r * m, 0, sizeof(double) * m);
        double sum = 0.0, comp = 0.0;      /* Neumaier summation of U */
        for (int ci = 0; ci < nc; ++ci) {
            int c = sel ? sel[ci] : ci;
            cview V;
            if ((rc = make_view(P, c, &V))) break;
            for (int s = 0; s < V.k; ++s) V.p[s] = pv[V.ids[s]];
            double PT, PF, dF[MAX_SUPPORT];
            if ((rc = constraint_cop(&V, &PT, &PF, dF))) break;
            double wc = w ? w[(size_t)r * C + c] : 1.0;
            if (unsat) unsat[(size_t)r * C + c] = PF;
            if (sat) sat[(size_t)r * C + c] = PT;
            double term = wc * PF;
            double t = sum + term;
            comp += fabs(sum) >= fabs(term) ? (sum - t) + term : (term - t) + sum;
            sum = t;
            for (int s = 0; s < V.k; ++s) {
                int id = V.ids[s];
                double g = wc * dF[s];                  /* dU/dp of this variable */
                if (id < n) {
                    double ga = g * -0.5;               /* dp/da = -1/2 */
                    if (grad_a) grad_a[(size_t)r * n + id] += ga;
                    if (absg_a) absg_a[(size_t)r * n + id] += fabs(ga);
                } else {
                    int k = id - n;
                    for (int64_t e = P->atom_ptr[k]; e < P->atom_ptr[k + 1]; ++e) {
                        double gb = g * dz[k] * P->atom_coef[e];   /* dp/db_j = dp/dz q_j */
                        int j = P->atom_var[e];
                        if (grad_b) grad_b[(size_t)r * m + j] += gb;
                        if (absg_b) absg_b[(size_t)r * m + j] += fabs(gb);
                    }
                }
            }
        }
        U[r] = sum + comp;
    }
    free(pv);
    free(dz);
    return rc;
}

/* Rounding x_i = True iff a_i < 0, then the exact check of every constraint.
 * sat_bits [R][ceil(C/32)]: bit c%32 of word c/32 set iff constraint c is satisfied. */
int oracle_check(const oproblem *P, int R, const float *a, const float *b, int8_t *x,
                 uint32_t *sat_bits, int32_t *n_unsat, int32_t *verdict)
{
    int n = P->n_bool, m = P->n_real, C = P->n_cons, nw = (C + 31) / 32;
    int8_t *truth = (int8_t *)malloc((size_t)(n + P->n_atoms) + 1);
    if (!truth) return -2;
    for (int r = 0; r < R; ++r) {
        const float *ar = a + (size_t)r * n, *br = b + (size_t)r * m;
        for (int i = 0; i < n; ++i) {
            truth[i] = ar[i] < 0.0f ? 1 : 0;
            if (x) x[(size_t)r * n + i] = truth[i] ? -1 : 1;
        }
        for (int k = 0; k < P->n_atoms; ++k) truth[n + k] = (int8_t)atom_true_at(P, k, br);
        uint32_t *bits = sat_bits + (size_t)r * nw;
        memset(bits, 0, sizeof(uint32_t) * nw);
        int cnt = 0;
        for (int c = 0; c < C; ++c) {
            cview V;
            if (make_view(P, c, &V)) { free(truth); return ORC_ELIMIT; }
            for (int s = 0; s < V.k; ++s) V.val[s] = truth[V.ids[s]];
            int v = eval3(&V);
            if (v == 1) bits[c >> 5] |= 1u << (c & 31); else ++cnt;
        }
        n_unsat[r] = cnt;
        verdict[r] = cnt == 0 ? 1 : 0;
    }
    free(truth);
    return ORC_OK;
}

/* Feasible set of the projection (Def. "Projection", Prop. "qp"): the box [-1,1]^n x
 * [lo, hi] and, when unit_proj is set, every unit atomic constraint (a constraint that is a
 * single atom literal, no propositional variable) as the closed half-space it asks for. A
 * half-space is shifted inward by delta = 1e-6 (|q0| + sum_j |q_j| max(|lo_j|, |hi_j|)) so
 * that its projected point satisfies the atom after rounding to float32; single-variable
 * ones are plain bounds and get no shift. Returns the number of half-spaces found. */
typedef struct { int n; int *ptr; int *var; double *coef; double *rhs; double *inv; } ohs;

static void find_units(const oproblem *P, const double *lo0, const double *hi0, double *lo, double *hi, ohs *H)
{
    int n = P->n_bool;
    H->n = 0;
    H->ptr = (int *)malloc(sizeof(int) * (size_t)(P->n_cons + 1));
    int64_t cap = P->atom_ptr[P->n_atoms] + 1;
    H->var = (int *)malloc(sizeof(int) * (size_t)cap);
    H->coef = (double *)malloc(sizeof(double) * (size_t)cap);
    H->rhs = (double *)malloc(sizeof(double) * (size_t)(P->n_cons + 1));
    H->inv = (double *)malloc(sizeof(double) * (size_t)(P->n_cons + 1));
    H->ptr[0] = 0;
    for (int j = 0; j < P->n_real; ++j) { lo[j] = lo0[j]; hi[j] = hi0[j]; }
    for (int c = 0; c < P->n_cons; ++c) {
        if (P->con_kind[c] != K_CLAUSE && P->con_kind[c] != K_AND) continue;
        if (P->con_ptr[c + 1] - P->con_ptr[c] != 1) continue;
        int lit = P->con_lit[P->con_ptr[c]];
        if ((lit >> 1) < n) continue;
        int k = (lit >> 1) - n;
        int op = P->atom_op[k];
        /* the constraint asks q.y <= q0 (or its strict / reversed / negated variant):
         * write the closed half-space as s q.y <= s q0 */
        double s = (op == O_GE || op == O_GT) ? -1.0 : 1.0;
        if (lit & 1) s = -s;
        int64_t e0 = P->atom_ptr[k], e1 = P->atom_ptr[k + 1];
        if (e1 - e0 == 1) {
            int j = P->atom_var[e0];
            double q = s * P->atom_coef[e0], bnd = s * P->atom_rhs[k] / q;
            double nlo = lo[j], nhi = hi[j];
            if (q > 0) { if (bnd < nhi) nhi = bnd; } else { if (bnd > nlo) nlo = bnd; }
            if (nlo <= nhi) { lo[j] = nlo; hi[j] = nhi; }
            continue;
        }
        int t = H->n, base = H->ptr[t];
        double scale = fabs(P->atom_rhs[k]), q2 = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            int j = P->atom_var[e];
            double m = fabs(lo0[j]) > fabs(hi0[j]) ? fabs(lo0[j]) : fabs(hi0[j]);
            scale += fabs(P->atom_coef[e]) * m;
            H->var[base + (e - e0)] = j;
            H->coef[base + (e - e0)] = s * P->atom_coef[e];
            q2 += P->atom_coef[e] * P->atom_coef[e];
        }
        H->rhs[t] = s * P->atom_rhs[k] - 1e-6 * scale;
        H->inv[t] = 1.0 / q2;
        H->ptr[t + 1] = base + (int)(e1 - e0);
        H->n = t + 1;
    }
}

static void free_units(ohs *H) { free(H->ptr); free(H->var); free(H->coef); free(H->rhs); free(H->inv); }

/* Euclidean projection of y onto box x half-spaces by Dykstra's alternating projections,
 * iterated until a whole sweep moves nothing by more than 1e-13 (1 + |y|). */
static void dykstra(double *y, int m, const double *lo, const double *hi, const ohs *H)
{
    if (H->n == 0) {
        for (int j = 0; j < m; ++j) y[j] = y[j] < lo[j] ? lo[j] : (y[j] > hi[j] ? hi[j] : y[j]);
        return;
    }
    double *pb = (double *)calloc((size_t)m + 1, sizeof(double));
    double *ph = (double *)calloc((size_t)H->ptr[H->n] + 1, sizeof(double));
    for (int sweep = 0; sweep < 1000000; ++sweep) {
        int moved = 0;
        for (int t = 0; t < H->n; ++t) {
            double viol = -H->rhs[t];
            for (int e = H->ptr[t]; e < H->ptr[t + 1]; ++e) viol += H->coef[e] * (y[H->var[e]] + ph[e]);
            double sh = viol > 0.0 ? viol * H->inv[t] : 0.0;
            for (int e = H->ptr[t]; e < H->ptr[t + 1]; ++e) {
                int j = H->var[e];
                double z = y[j] + ph[e], yp = z - sh * H->coef[e];
                if (fabs(yp - y[j]) > 1e-13 * (1.0 + fabs(yp))) moved = 1;
                ph[e] = z - yp;
                y[j] = yp;
            }
        }
        for (int j = 0; j < m; ++j) {
            double z = y[j] + pb[j], yp = z < lo[j] ? lo[j] : (z > hi[j] ? hi[j] : z);
            if (fabs(yp - y[j]) > 1e-13 * (1.0 + fabs(yp))) moved = 1;
            pb[j] = z - yp;
            y[j] = yp;
        }
        if (!moved) break;
    }
    free(pb);
    free(ph);
}

/* Projected gradient step (Eq. "pg1"/"pg2") and the gradient map norm ||g||^2
 * (Eq. "grad_map") per point. Comparisons keep NaN as NaN in the clamp. */
int oracle_pgd(const oproblem *P, int R, const float *a, const float *b, const float *ga,
               const float *gb, double eta_a, double eta_b, const double *lo0, const double *hi0,
               int unit_proj, double *a_out, double *b_out, double *gsq)
{
    int n = P->n_bool, m = P->n_real;
    double *lo = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    double *hi = (double *)malloc(sizeof(double) * ((size_t)m + 1));
    ohs H = {0, 0, 0, 0, 0, 0};
    if (unit_proj) {
        find_units(P, lo0, hi0, lo, hi, &H);
    } else {
        for (int j = 0; j < m; ++j) { lo[j] = lo0[j]; hi[j] = hi0[j]; }
    }
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) {
            double x = (double)a[(size_t)r * n + i];
            double y = x - eta_a * (double)ga[(size_t)r * n + i];
            double p = y < -1.0 ? -1.0 : (y > 1.0 ? 1.0 : y);
            a_out[(size_t)r * n + i] = p;
            double g = (x - p) / eta_a;
            acc += g * g;
        }
        double *y = b_out + (size_t)r * m;
        for (int j = 0; j < m; ++j) y[j] = (double)b[(size_t)r * m + j] - eta_b * (double)gb[(size_t)r * m + j];
        dykstra(y, m, lo, hi, &H);
        for (int j = 0; j < m; ++j) {
            double g = ((double)b[(size_t)r * m + j] - y[j]) / eta_b;
            acc += g * g;
        }
        gsq[r] = acc;
    }
    int nh = H.n;
    if (unit_proj) free_units(&H);
    free(lo);
    free(hi);
    return nh;
}

/* Projection of one point onto D alone (for pinning the projection). */
int oracle_project(const oproblem *P, const double *y_in, const double *lo0, const double *hi0,
                   int unit_proj, double *y_out, double *lo_out, double *hi_out)
{
    int m = P->n_real;
    ohs H = {0, 0, 0, 0, 0, 0};
    if (unit_proj) {
        find_units(P, lo0, hi0, lo_out, hi_out, &H);
    } else {
        for (int j = 0; j < m; ++j) { lo_out[j] = lo0[j]; hi_out[j] = hi0[j]; }
    }
    for (int j = 0; j < m; ++j) y_out[j] = y_in[j];
    dykstra(y_out, m, lo_out, hi_out, &H);
    int nh = H.n;
    if (unit_proj) free_units(&H);
    return nh;
}

/* ERWA update of Alg. "CLS with Annealing" for one sigma-level t (1-based):
 * u_c = [c violated]; h_c = rho h_c + u_c; every tau levels w_c *= gamma^h_c and h_c = 1;
 * optionally renormalize w to sum C. */
void oracle_erwa(int R, int C, const uint32_t *sat_bits, int t, double rho, double gamma,
                 int tau, int normalize, double *h, double *w)
{
    int nw = (C + 31) / 32;
    for (int r = 0; r < R; ++r) {
        double tot = 0.0;
        for (int c = 0; c < C; ++c) {
            int viol = !((sat_bits[(size_t)r * nw + (c >> 5)] >> (c & 31)) & 1u);
            size_t q = (size_t)r * C + c;
            h[q] = rho * h[q] + (double)viol;
            if (t % tau == 0) {
                w[q] = w[q] * pow(gamma, h[q]);
                h[q] = 1.0;
            }
            tot += w[q];
        }
        if (normalize && t % tau == 0)
            for (int c = 0; c < C; ++c) w[(size_t)r * C + c] *= (double)C / tot;
    }
}
