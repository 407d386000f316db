// Host-side set-up of the igaefie operator: geometry in Bezier form, the glued
// unknowns, the cluster and block-cluster trees, the near-field sparsity pattern
// and the small moment / transfer tables.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace ige {

struct Geometry {
    int P = 0;
    std::vector<PatchHdr> hdr;
    std::vector<double> brk, cp;
    double scale = 1.0;          // bounding-box size of the control net
    // edge partner: for (patch, edge) -> (patch', edge', reversed) or -1
    std::vector<std::array<int, 3>> partner;   // [P*4]
    GeomView view() const { return GeomView{hdr.data(), brk.data(), cp.data()}; }
};

// Validate NURBS input, convert to rational Bezier spans, match the patch edges.
void build_geometry(Geometry &G, int P, const int *degree, const int *n_ctrl, const double *knots,
                    const double *ctrl);

// Gauss-Legendre rule on [0,1] (n points, ascending).
void gauss_legendre01(int n, double *x, double *w);

// Chebyshev points of the first kind on [0,1] and Lagrange polynomials on them
// (barycentric form).
void chebyshev01(int q, double *x);
void lagrange_bary(int q, const double *xn, double s, double *L);

struct Discretisation {
    int P, p, m, n, nb, N;
    int scalar = 0;             // 1: scalar single layer (tensor B-splines of degree p per patch, not glued)
    std::vector<int32_t> dof;   // [P][2][nb][nb]
    std::vector<int8_t> sgn;
    // per unknown up to two incarnations (patch, comp, i1, i2, sign); patch -1 = none
    std::vector<std::array<int32_t, 5>> inc;   // [N*2]
    // 1-D Bezier extraction of the uniform p-open splines, per element:
    // ext_p[e][t][k]: Bernstein(degree p) coefficient k of b^p_{e+t} on element e;
    // ext_q[e][t][k]: Bernstein(degree p-1) coefficient k of b^{p-1}_{e+t}.
    std::vector<double> ext_p, ext_q;
};

void build_discretisation(Discretisation &D, const Geometry &G, int p, int m, int scalar = 0);

struct Partition {
    int L = 0;                    // leaf level
    int s = 1;                    // elements per leaf cluster side
    std::vector<std::array<int32_t, 3>> far;    // (level, target, source), sorted
    std::vector<std::array<int32_t, 2>> near;   // (target leaf, source leaf), sorted
    std::vector<double> diam;                   // [L+1] largest bounding-ball diameter per level
};

// Algorithm 1 from all ordered patch pairs with the admissibility condition
// max diam <= eta dist; kappa_cap > 0 adds kappa * max diam <= kappa_cap
void build_partition(Partition &T, const Geometry &G, const Discretisation &D, double eta, int leaf_depth, double kappa,
                     double kappa_cap);

// Near field as dense blocks over leaf function slots.  The functions whose
// support meets a leaf cluster (2^d x 2^d elements, degree p) are numbered by a
// leaf-local slot: component 0 has (W) x (W-1) functions, component 1 (W-1) x (W),
// W = 2^d + p, so nF = 2 W (W-1) slots per leaf.  The operator is complex
// symmetric, so one block is stored per unordered near leaf pair (t <= s); the
// block of (s, t) is its transpose.  Block entries are in glued unknowns (signs
// folded in).  The product writes per-block partial results, which a fixed-order
// reduction sums per unknown (deterministic).
struct NearBlocks {
    int W = 0, nF = 0;
    int nch = 1, rc = 0;                 // row chunks per block, rows per chunk
    std::vector<int32_t> pair;           // [nblk][2] (target leaf, source leaf), target <= source
    std::vector<int32_t> leafdof;        // [nleaf][nF] glued unknown, -1 = no function
    std::vector<int8_t> leafsgn;         // [nleaf][nF]
    std::vector<int64_t> red_ptr;        // [N+1]
    std::vector<int32_t> red_idx;        // partial-result slots, in block order
    int64_t nblk() const { return (int64_t)pair.size() / 2; }
    // partial-result slots: rows [nblk][nF], then columns [nblk][nch][nF]
    int64_t nslots() const { return nblk() * nF * (1 + nch); }
};
constexpr int kMaxLeafSlots = 1024;
__host__ __device__ inline int leaf_slot(int W, int a, int i1, int i2)
{
    return a == 0 ? i2 * W + i1 : W * (W - 1) + i2 * (W - 1) + i1;
}
void build_near_blocks(NearBlocks &B, const Discretisation &D, const Partition &T, int nch);

// The same near-field matrix stored once per distinct entry (used by the product of
// one column).  Every glued unknown is owned by one leaf (the leaf of the last element
// of its support, at its first incarnation).  An entry (i, j) lives in the owner block
// (own(i), own(j)) if own(i) <= own(j), else as (j, i) in (own(j), own(i)) (the matrix
// is complex symmetric).  An off-diagonal owner block is split into dense
// rectangles: its rows grouped by the set of source leaves whose slots give their
// columns, each group times the union of those columns, so every stored entry is a
// distinct nonzero.  A diagonal owner block is one dense square over its unknowns, of
// which the product reads the upper triangle.  The values are summed from the leaf-pair
// blocks (k_near_merge) in a fixed order.
struct NearCompact {
    std::vector<int32_t> nr, nc;       // [nsub] rows, columns of each rectangle
    std::vector<int8_t> sym;           // [nsub] 1: diagonal square (upper triangle used)
    std::vector<int64_t> val;          // [nsub] first value (row-major nr x ld, 256-byte aligned)
    std::vector<int32_t> ld;           // [nsub] row stride: nc rounded up to 4 (64-byte rows)
    std::vector<int64_t> lst;          // [nsub] first entry in idx: nr rows then nc columns
    std::vector<int32_t> idx;          // glued unknowns
    int64_t nval = 0;                  // stored values (full squares, padded rows)
    int64_t distinct = 0;              // distinct entries (upper triangles of the squares)
    int maxn = 0;                      // largest nr or nc
    // work items of the product: rows [r0, r1) of one rectangle; partial results at
    // part[w]: (r1 - r0) row sums, then nc column sums
    std::vector<int32_t> wsub, wr0, wr1;
    std::vector<int64_t> wpart;
    std::vector<int32_t> worder;       // launch order of the work items
    int64_t nnarrow = 0;               // leading work items of at most 128 columns
    int64_t npart = 0;
    std::vector<int64_t> red_ptr;      // [N+1] partial results of every unknown, ascending
    std::vector<int32_t> red_idx;
    // merge tables: leaf slots holding each unknown (leaf * nF + slot), ascending, and
    // per leaf its near partners (both orders) with code = 2 * block + (leaf > partner)
    std::vector<int32_t> occ_ptr, occ;
    std::vector<int32_t> np_ptr, np_leaf, np_code;
    int64_t nsub() const { return (int64_t)nr.size(); }
};
void build_near_compact(NearCompact &C, const Discretisation &D, const Partition &T, const NearBlocks &B,
                        int rows_per_item);

// singular element pairs inside the near field: (test element, trial element,
// kind 1 identical / 2 edge / 3 vertex, frame code test, frame code trial)
// Only pairs whose leaf pair is stored (leaf(e) <= leaf(f)) are kept; blk is the
// index of that block.
struct SingularPair {
    int32_t e, f;
    int32_t kind;
    int32_t fa, fb;   // frame code: bit0 = o1, bit1 = o2, bit2 = swap (see kernels)
    int32_t blk;
};
void build_singular_pairs(std::vector<SingularPair> &S, std::vector<double> &corners, const Geometry &G,
                          const Discretisation &D, const Partition &T, const NearBlocks &B);

// 1-D moment tables of the leaf clusters and transfer matrices
// q: the largest degree of the levels; the upward and downward passes (moments of
// the leaves, M2M, L2L, L2P) run in it on every level.  A level l of smaller degree
// q_l takes its moments by the exact restriction R_l[n][m] = L^{q_l}_m(x^q_n) of the
// degree-q moments (a degree-q_l Lagrange polynomial is reproduced by degree-q
// interpolation) and gives its local expansions back through R_l^T.
struct FarTables {
    int q, Q1, rowlen;            // rowlen = s + p
    bool varq = false;            // some level's degree differs from q
    std::vector<int> ql;               // [L+1] degree of each level
    std::vector<double> Mp, Mq, Mdp;   // [2^L][Q1][rowlen]
    std::vector<double> T0, T1;        // [Q1][Q1]: T_c[n][m] = L_m((x_n + c)/2)
    std::vector<double> xn;            // nodes
    std::vector<double> xnl;           // [L+1][kMaxQ1] nodes of each level's degree
    std::vector<double> R;             // [L+1][Q1][Q1] restriction (columns m <= q_l used)
};
void build_far_tables(FarTables &F, const Discretisation &D, const Partition &T, const std::vector<int> &ql);

}  // namespace ige
