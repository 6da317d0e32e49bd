// Internal layout of a compiled instance (host compiler <-> HIP kernels).
//
// HBM layout (all arrays device-resident, read-only after xbdd_compile):
//  * Diagram shapes ("templates"): constraints whose reduced ordered BDDs are identical up to
//    renaming of their support variables share one node table. A node is 8 bytes
//    {slot, hi, lo, pad} (u16 each); nodes are in topological order with the root at index
//    0; child index n_nodes is the True terminal, n_nodes+1 the False terminal. Slots index
//    the constraint's sorted support (Booleans first, then atoms).
//  * Buckets: constraints of one template, in original order, padded to a multiple of 64
//    "positions" so that a 64-lane wavefront never straddles two templates. The support ids
//    of a bucket are stored slot-major (sup[sup_base + s*n_pos + local]) so that lanes
//    working on consecutive constraints read consecutive words.
//  * Atoms in "<=" form: ">=" / ">" atoms are stored negated (exact in floating point), with
//    FP64 coefficients and right-hand side, the smoothing scale 1/(sqrt(2)|q|), and a
//    strictness flag for the exact test.
#pragma once
#include <cstdint>
#include <vector>

#include "../../include/fsmt.h"

namespace fsmt {

struct TplInfo {
    int32_t node_off;   // first node in the node table
    int32_t n_nodes;    // decision nodes (terminals excluded)
    int32_t n_slots;    // support size
    int32_t n_bslots;   // Boolean slots (slots [0, n_bslots) are Booleans)
    int32_t root;       // 0, or n_nodes / n_nodes+1 for constant constraints
    int32_t lev_off;    // level starts: lev[lev_off + s] = first node of slot s (s <= n_slots)
    int32_t pad[2];     // pad[0]: pair count L of a pair disjunction, -1 a guarded disjunction, else 0
};

// A diagram is "big" when its per-lane message columns would take more than 40 KB of LDS
// per wavefront (four such wavefronts fill a compute unit's LDS); big diagrams are
// evaluated level by level, one wavefront per (constraint, restart), instead of one lane
// per constraint. Every diagram within the register bounds below is under the limit.
constexpr int64_t kBigDiagramBytes = 40960;
// Bounds of the largest register-resident message store: node messages take nodes + 3
// registers (two terminals and a spare), which must stay within one 32-register tuple
// for indexed register access.
constexpr int kLargeMaxNodes = 29, kLargeMaxSlots = 24;
// Pair disjunctions OR_i (x_{2i} XOR x_{2i+1}) OR a_0 OR ... OR a_{T-1} (index bits that
// differ, or one of T atoms) are evaluated in closed form (see pair_eval) up to these sizes;
// their templates carry L in TplInfo::pad[0] / BucketInfo::pad (0: generic diagram).
constexpr int kPairMaxL = 10, kPairMaxT = 4;
// Guarded disjunctions: diagrams whose first k <= kGdMaxSel slots ("selectors") route every
// assignment of them either to a terminal or to a chain in which each node has one edge to
// the True terminal, i.e. to a disjunction of literals over the later slots (a clause, an
// ITE over one or two Booleans of such clauses). The false-terminal mass is then
//   F = sum_g pi_g prod_{s in S_g} l_s,   pi_g = prod_{i < k} P[slot i = g_i],
// with l_s = P[literal s False], evaluated in closed form (see gd_eval) for supports of at
// most kGdMaxSlots slots.
// Selectors are Boolean slots; the evaluation keeps every slot in registers, so the family is
// bounded to kGdMaxBool Boolean and kGdMaxAtoms atom slots, each atom with an inline record.
constexpr int kGdMaxSel = 2, kGdMaxBool = 4, kGdMaxAtoms = 8;
struct GdInfo {
    uint32_t mask[4];   // per selector assignment g (bit i = value of selector i): slots of its
                        // disjunction; bit 31 set: the assignment reaches the True terminal
    uint32_t neg;       // slots whose literal is negated (False iff the variable is True)
    int32_t k;          // selector slots (slots 0 .. k-1)
    uint32_t same_vars; // bit j: atom slot j has the variables of atom slot j-1 in every constraint
                        // of the template (their values are read once, their gradients summed)
    uint32_t same_lin;  // bit j: ... and the same coefficients (q.y is computed once)
    // Separable (k = 2, no other Boolean slot, no assignment reaching True): selector i's
    // value v alone picks the atoms S_{i,v} of the disjunction, the four sets are disjoint
    // and each has at most two atoms, so
    //   F = (P[s0 F] L(S_{0,0}) + P[s0 T] L(S_{0,1})) (P[s1 F] L(S_{1,0}) + P[s1 T] L(S_{1,1})),
    // L(S) the product of S's literal-false probabilities. sep_slots holds the atom slots of
    // S_{0,0}, S_{0,1}, S_{1,0}, S_{1,1}, two 4-bit fields per group (kGdMaxAtoms: none).
    uint32_t sep;
    uint32_t sep_slots;
    uint32_t pad[6];
};
// Closed-form levels a kernel carries (chosen by the host from the instances of a launch, so
// that a kernel holds only the register footprint it needs): 0 none; 1 guarded disjunctions
// of at most one Boolean and two atom slots (clauses, feasibility ITEs); 2 also two Boolean
// selectors over up to kGdMaxAtoms atoms; 3 every guarded disjunction and the pair
// disjunctions.
inline int gd_level_of(int n_bslots, int n_aslots) { return (n_bslots <= 1 && n_aslots <= 2) ? 1 : n_bslots <= 2 ? 2 : 3; }
// Unit-atom half-spaces that share no variable, each over at most this many distinct
// variables, are projected onto in closed form (project_dykstra) instead of by sweeps.
constexpr int kSeparableRowMax = 4;
inline bool big_diagram(int n_nodes, int n_slots) {
    const int64_t ss = n_slots > 1 ? n_slots : 1;
    return (2 * ((int64_t)n_nodes + 2) + 4 * ss) * 64 * 4 > kBigDiagramBytes;
}

struct BucketInfo {
    int32_t tpl;        // template id
    int32_t pos_begin;  // first position (multiple of 64)
    int32_t n_pos;      // positions, a multiple of 64 (>= constraints in the bucket)
    int32_t n_con;      // real constraints in the bucket
    int64_t sup_base;   // offset of the bucket's support block (n_slots * n_pos ids)
    int64_t arec_base;  // offset of the bucket's inline atom records, or -1
    // copy of the template record (one scalar load serves the whole wave)
    int32_t node_off, n_nodes, n_slots, n_bslots, root;
    int32_t lev_off;    // level starts of the template
    int32_t big;        // 1: big diagram (level-synchronous kernel), 0: one lane per constraint
    int32_t pad;        // closed-form family: L > 0 pair disjunction with L pairs, -1 guarded
                        // disjunction (record in gd[tpl]), 0 the generic message passing
};

// Inline atom record (atoms with at most two variables whose "<=" coefficients and
// right-hand side are exact in float32): one coalesced 32-byte load per (position, atom
// slot) replaces the CSR indirection. Records are stored per bucket, atom-slot-major:
// arec[arec_base + (slot - n_bslots) * n_pos + local]. Promoting the float32 values to
// FP64 gives exactly the stored atom, so the exact test is unchanged.
struct AtomRec {
    int32_t v0, v1;     // real variables (v1 unused when nnz == 1)
    float c0, c1;       // coefficients in "<=" form
    float rhs;          // right-hand side in "<=" form
    float scale;        // 1/(sqrt(2)|q|)
    int32_t atom;       // atom id
    uint32_t flags;     // bit 0 strict, bit 1 two variables
};

struct Node {
    uint16_t slot, hi, lo, pad;
};

// Guarded disjunctions stream slim atom records: in every member of such a template, atom
// slot j has the same coefficients, scale and flags (kept once per template in GdForm), so
// per (atom slot, position) only the variables and the right-hand side are stored, 12 bytes
// instead of the 32 of an AtomRec: slim[srec_base + j * n_pos + local]. The AtomRec copies
// stay for the exact check and the other passes.
struct SlimRec {
    int32_t v0, v1;   // real variables (v1 = v0 when the atom has one term)
    float rhs;        // right-hand side in "<=" form
};
struct GdForm {
    int64_t srec_base;             // offset of the template's bucket in the slim records
    uint32_t flags;                // bit j: atom slot j strict; bit 8 + j: two variables
    int32_t pad;
    float c0[kGdMaxAtoms], c1[kGdMaxAtoms], scale[kGdMaxAtoms];
};

struct DeviceTables {
    TplInfo *tpl = nullptr;
    Node *nodes = nullptr;
    BucketInfo *bucket = nullptr;
    int32_t *bucket_start = nullptr;  // [n_buckets+1] position prefix
    int32_t *task_bucket = nullptr;   // [n_pos/64] bucket of each 64-position group
    AtomRec *arec = nullptr;          // inline atom records
    int32_t *pos_con = nullptr;       // [n_pos] original constraint id or -1 (padding)
    int32_t *sup = nullptr;           // support ids, slot-major per bucket
    int32_t *con_bucket = nullptr;    // [C]
    int32_t *con_local = nullptr;     // [C] index inside its bucket
    int32_t *atom_ptr = nullptr;      // [A+1]
    int32_t *atom_var = nullptr;      // [nnz]
    double *atom_coef = nullptr;      // [nnz] ("<=" form)
    double *atom_rhs = nullptr;       // [A]   ("<=" form)
    double *atom_scale = nullptr;     // [A]   1/(sqrt(2)|q|)
    uint8_t *atom_strict = nullptr;   // [A]
    int32_t *lev = nullptr;           // per template: n_slots + 1 level starts
    int32_t *big_pos = nullptr;       // positions of the constraints in big buckets
    GdInfo *gd = nullptr;             // [n_tpl] guarded-disjunction records (k = -1: not one)
    GdForm *gdf = nullptr;            // [n_tpl] their per-slot coefficients, scales and flags
    SlimRec *srec = nullptr;          // slim atom records of the guarded-disjunction buckets
    float *real_lo = nullptr;         // [m] box of D (tightened by single-variable unit atoms)
    float *real_hi = nullptr;         // [m]
    int32_t *hs_ptr = nullptr;        // [H+1] half-spaces of D: q.y <= rhs (multi-variable unit atoms)
    int32_t *hs_var = nullptr;
    float *hs_coef = nullptr;
    float *hs_rhs = nullptr;          // [H] q0 - delta
    float *hs_inv = nullptr;          // [H] 1 / |q|^2
    int32_t *hs_cstart = nullptr;     // [K+1] colour classes: half-spaces of a class share no variable
};

}  // namespace fsmt

struct fsmt_xbdd {
    int device = 0;
    int n_bool = 0, n_real = 0, n_atoms = 0, n_cons = 0;
    int n_tpl = 0, n_buckets = 0, n_pos = 0;
    int max_nodes = 0, max_slots = 0;
    int small_max_nodes = 0, small_max_slots = 0;   // over templates evaluated one lane per constraint
    int big_max_nodes = 0, big_max_slots = 0;       // over big templates
    int n_big = 0;                                  // constraints in big buckets
    int64_t total_nodes = 0, nnz = 0, table_bytes = 0;
    int n_box_units = 0, n_hs = 0, hs_nnz = 0, n_hs_colors = 0;
    int hs_separable = 0;   // one colour class, rows of at most kSeparableRowMax distinct variables
    int64_t n_pair = 0;               // constraints evaluated as pair disjunctions (closed form)
    int64_t n_gd = 0;                 // constraints evaluated as guarded disjunctions (closed form)
    int64_t n_gd_sep = 0;             // ... of which separable (GdInfo::sep)
    int gd_level = 0;                 // largest closed-form level of its guarded disjunctions (1..3)
    bool lds_messages = false;   // FSMT_MSG_LDS: never the register-resident message variants
    bool all_inline = false;     // every atom slot of every bucket has an inline record
    std::vector<fsmt::TplInfo> h_tpl;
    std::vector<fsmt::BucketInfo> h_bucket;
    std::vector<int32_t> h_bucket_start;
    std::vector<fsmt::Node> h_nodes;
    std::vector<int32_t> h_sup, h_con_bucket, h_con_local;
    bool host_only = false;
    fsmt::DeviceTables d;
    std::vector<void *> allocations;
};

namespace fsmt {
// error reporting shared by the ABI entry points
fsmt_status set_error(fsmt_status code, const char *fmt, ...);
void clear_error();
}  // namespace fsmt
