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
    std::vector<int32_t> dof;   // [P][2][nb][nb]
    std::vector<int8_t> sgn;
    // per unknown up to two incarnations (patch, comp, i1, i2, sign); patch -1 = none
    std::vector<std::array<int32_t, 5>> inc;   // [N*2]
    // 1-D Bezier extraction of the uniform p-open splines, per element:
    // ext_p[e][t][k]: Bernstein(degree p) coefficient k of b^p_{e+t} on element e;
    // ext_q[e][t][k]: Bernstein(degree p-1) coefficient k of b^{p-1}_{e+t}.
    std::vector<double> ext_p, ext_q;
};

void build_discretisation(Discretisation &D, const Geometry &G, int p, int m);

struct Partition {
    int L = 0;                    // leaf level
    int s = 1;                    // elements per leaf cluster side
    std::vector<std::array<int32_t, 3>> far;    // (level, target, source), sorted
    std::vector<std::array<int32_t, 2>> near;   // (target leaf, source leaf), sorted
};

void build_partition(Partition &T, const Geometry &G, const Discretisation &D, double eta, int leaf_depth);

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
struct FarTables {
    int q, Q1, rowlen;            // rowlen = s + p
    std::vector<double> Mp, Mq, Mdp;   // [2^L][Q1][rowlen]
    std::vector<double> T0, T1;        // [Q1][Q1]: T_c[n][m] = L_m((x_n + c)/2)
    std::vector<double> xn;            // nodes
};
void build_far_tables(FarTables &F, const Discretisation &D, const Partition &T, int q);

}  // namespace ige
