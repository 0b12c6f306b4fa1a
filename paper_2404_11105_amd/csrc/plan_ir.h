// plan_ir.h — the compact plan descriptor read by the count kernel.
//
// A plan binds pattern vertices level by level (section 5.1: a
// materialisation order of vertices and an exploration order of edges).
// Level 0 is the start vertex (its images are the roots, Algorithm 2's
// "init A^{p.start}").  Levels 1..e-1 are enumerated: each partial match is
// extended by every candidate of the next level (Algorithm 2, Explore).  The
// trailing vertices are a leaf group: they have no arcs among themselves, so
// once levels 0..e-1 are bound their candidate sets are fixed and the number
// of injective completions is computed from set sizes instead of being
// enumerated (section 5.3, counting by multiplying candidate-set sizes, made
// exact for overlapping sets by inclusion-exclusion over set partitions).
//
// Candidates of a level satisfy:
//   * one membership per constraint (j, dir): x in out(phi(v_j)) for dir 0,
//     x in in(phi(v_j)) for dir 1 (Definition 2.2 edge constraints, with the
//     direction check of Algorithm 2's out_arcs / in_arcs choice);
//   * x != phi(v_j) for the levels j in `inj` (the visited marks of
//     Algorithm 2);
//   * out-degree >= dmin_out and in-degree >= dmin_in (the degree vertex
//     constraint, section 2, split into its two directions).
// A level with reuse = r takes its base from the candidates already found for
// level r under the same ancestors (section 5.2 intermediate-result reuse: an
// included constraint is materialised from the including one's result) and
// checks only the constraints in `extra`.
//
// Symmetry breaking (the symmetry destruction of the related-work section,
// made exact): with H the automorphisms of the pattern that map the
// conditioned vertices (the enumerated levels, plus the leaf when the leaf
// group is one vertex) onto themselves, H acts freely on the partial matches
// of those vertices and leaves the number of completions unchanged.  A
// stabiliser chain of H, taken in level order, gives conditions
// phi(v_j) < phi(v_i) (j earlier than i) that exactly one partial match of
// every H-orbit meets; the plan counts those and scales by |H| restricted to
// the conditioned vertices (sym_mult).  Only a lower bound arises per level:
// the largest image among the levels in `gt` (or, with the conditions
// reversed, phi(v_i) < phi(v_j), an upper bound: the smallest image).  Both
// directions are exact; which one enumerates less depends on the graph.
#pragma once
#include <stdint.h>

namespace xm {

constexpr int kMaxK = 7;          // pattern vertices
constexpr int kMaxCons = 12;      // constraints of one level (bidirected: 2 per earlier level)
constexpr int kMaxSig = 4;        // distinct leaf signatures
constexpr int kMaxLeaves = 6;     // vertices in the leaf group
constexpr int kMaxTerms = 96;     // inclusion-exclusion terms after merging
constexpr int kMaxBlocks = 6;     // blocks in one term
constexpr int kMaxMasks = 15;     // distinct signature masks the terms use
constexpr uint8_t kNoReuse = 0xFF;

struct LevelDesc {
    uint8_t n_cons;
    uint8_t reuse;                // kNoReuse or an enumerated level r >= 1
    uint8_t inj;                  // bit j: check x != phi(v_j)
    uint8_t deg_check;            // 1: check degree thresholds
    uint16_t extra;               // when reusing: bit c -> check constraint c
    uint16_t dir_mask;            // bit c = cons_dir[c] (packed copy for the kernel)
    uint8_t cons_lvl[kMaxCons];
    uint8_t cons_dir[kMaxCons];   // 0: out(phi(v_j)), 1: in(phi(v_j))
    uint32_t dmin_out, dmin_in;
    uint64_t lvl_bits;            // cons_lvl[c] at bits [3c, 3c+3) (packed copy)
    uint8_t gt;                   // bit j: phi(v_j) bounds the candidates (symmetry breaking)
    uint8_t lt;                   // 0: keep x > every bound; 1: keep x < every bound
    uint8_t pad[6];
};

struct Term {
    int32_t coef;                 // Moebius coefficient, merged
    uint8_t nb;                   // blocks
    uint8_t mask[kMaxBlocks];     // signature mask of each block (intersection of those sets)
    uint8_t pad;
};

struct PlanDesc {
    uint32_t k;                   // pattern vertices
    uint32_t e;                   // enumerated levels including the start vertex (1..k-1)
    uint32_t root_dout, root_din; // degree thresholds of the start vertex
    uint32_t seg_src;             // bit r: level r is a reuse source (track children)
    uint32_t n_sig;               // distinct leaf signatures (1..kMaxSig)
    uint32_t t;                   // leaves
    uint32_t linear;              // 1: one leaf -> the count is a plain sum of set sizes
    uint32_t n_terms;
    uint32_t sym_mult;            // >1: the plan counts one embedding per orbit of this size
    LevelDesc lvl[kMaxK];         // [1..e-1]
    LevelDesc sig[kMaxSig];       // leaf signatures (inj over levels < e)
    uint8_t sig_mult[kMaxSig];    // leaves per signature
    uint8_t order[kMaxK];         // level -> pattern vertex (reporting)
    uint8_t sym_fixes_root;       // 1: the symmetry group fixes the start vertex (root subsets stay exact)
    uint8_t root_share;           // s: only roots (stored ids) r with r mod 2^s = 2^s - 1 are tried (0: all)
    uint8_t pad2[3];
    Term terms[kMaxTerms];
    // Every signature mask M used by a term block, with the candidate test of
    // the intersection of those signatures' sets (union of their constraints):
    // the kernel measures |intersection over s in M of S_s| per partial match.
    // Masks whose tests coincide (the same union of constraints) share one
    // entry: mask_set[i] holds every mask M (bit M) that takes entry i's size.
    uint32_t n_masks;
    uint8_t mask_id[16];          // first mask of entry i (reporting)
    uint16_t mask_set[16];
    LevelDesc mdesc[kMaxMasks];
};

}  // namespace xm
