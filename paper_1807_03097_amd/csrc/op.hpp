// The assembled operator: host tables and device buffers, plus the kernel
// launchers that implement assembly, apply, right-hand side and GMRES steps.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <map>
#include <memory>
#include <vector>

#include "common.hpp"
#include "setup.hpp"

struct ige_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // geometries, operators and servers made on this context and not yet destroyed:
    // they use its device and stream, so the context outlives them
    std::atomic<int> users{0};
};

struct ige_geom_s {
    ige_ctx ctx = nullptr;
    ige::Geometry G;
};

namespace ige {

using cd = double2;   // complex double as (re, im)

// Device view of the operator, passed by value to kernels.
struct DevOp {
    int P, p, m, n, nb, N, nl, L, s, SL;   // SL = 2^L leaf clusters per patch side
    int scalar;                // 1: scalar single layer (one component: value times |J| in slot 3)
    double cdiv;               // factor of the slot-3 term: -kappa^-2 (EFIE divergence), 1 (scalar)
    int q, Q1, Q, g, G2, gs;
    double kappa, h, scale_tol;
    GeomView geo;
    const int32_t *dof;
    const int8_t *sgn;
    const double *ext_p, *ext_q;       // [n][p+1][p+1], [n][p][p]
    const double *gx, *gw, *sx, *sw;   // regular / singular 1-D Gauss rules on [0,1]
    // element data at the regular Gauss points
    const double *eX;      // [E][3][G2]
    const double *ePsi;    // [E][4][nl][G2]  weight * (phi_hat d_aF (3 comps), div phi_hat)
    const double *ePsiF;   // the same values in matrix-core operand order, see k_element_data
    const double *eC;      // [E][4][3] element corners
    // near field: dense blocks over leaf function slots
    int W, nF, nch, rc;
    int64_t nblk;
    const int32_t *bpair;     // [nblk][2]
    double2 *bval;            // [nblk][nF][nF]
    const int32_t *leafdof;   // [nleaf][nF]
    const int8_t *leafsgn;    // [nleaf][nF]
    const int64_t *red_ptr;   // [N+1]
    const int32_t *red_idx;
    // element pairs with a shared corner: the list, their blocks [nsing][nl][nl]
    // (assembly scratch) and per (block, test element of the target leaf) the range of
    // list entries [nblk][s^2 + 1]
    const SingularPair *sing;
    double2 *sblk;
    const int32_t *sing_ptr;
    // cluster tree
    const int64_t *lvl_off;   // [L+2] first global cluster id of each level
    const double *nodeX;      // [NC][3][Q]
    const double *nodeT;      // [NC][6][Q]  d_uF (3), d_vF (3)
    const double2 *sctab;     // [256] (cos, sin)(j pi/128) / (4 pi), for the table-driven kernel evaluation
    const double *xn;         // [Q1] Chebyshev nodes of degree q (the largest level degree)
    // degree per level (variable order): varq = 1 when some level's degree ql[l] < q;
    // its nodes xnl [L+1][kMaxQ1] and the restriction Rl [L+1][Q1][Q1] from degree q
    int varq;
    int ql[kMaxLev];
    const double *xnl, *Rl;
    const double *T0, *T1;    // [Q1][Q1]
    const double *Mp, *Mq, *Mdp;   // [SL][Q1][rowlen]
    int rowlen;
    const int32_t *inc;       // [N][2][5]
    int *err;                 // assembly consistency counter (entries outside the pattern)
};

// Device view of the near field stored once per distinct entry (NearCompact).
struct NearCmpView {
    int64_t nsub, nwork;
    const int32_t *nr, *nc, *ld;
    const int8_t *sym;
    const int64_t *val_off, *lst;
    const int32_t *idx;
    double2 *val;
    const int4 *work;          // (rectangle, r0, r1, 0)
    const int64_t *wpart;      // first partial result of each work item
    const int32_t *order;      // launch order of the work items
    const int32_t *occ_ptr, *occ, *np_ptr, *np_leaf, *np_code;
};

struct M2LWork {
    int32_t tgt;      // global cluster id
    int32_t beg, end; // range in the partner array
};

}  // namespace ige

struct ige_op_s {
    ige_ctx ctx = nullptr;
    ige_params prm{};
    bool assembled = false;   // false: planned on the host only
    ige::Discretisation D;
    ige::Partition T;
    ige::FarTables F;
    int64_t nnz = 0;
    int64_t nsing = 0;
    double assemble_ms = 0.0;
    int profiling = 0;                 // 0 off, 1 every stage boundary, 2 the block pass and coupling kernel only
    int prof_level_rec = 0;            // level of the recorded applies
    static constexpr int kProfSlots = 256;
    static constexpr int kProfEv = 13;
    std::vector<hipEvent_t> prof_ev;   // [kProfSlots][kProfEv] stage boundary events
    hipStream_t aux = nullptr;         // second stream: near-field product
    hipStream_t lst = nullptr;         // launch stream of the apply kernels (null: the context stream)
    hipStream_t gstream = nullptr;     // stream on which apply graphs are captured
    std::map<long long, int> tune;     // autotuned tile choices: (knob, columns, precision) -> value
    bool overlap = true;               // near field concurrent with the far field
    // coarsest level with far pairs (L + 1 if none): the upward pass stops there and
    // the downward pass starts there, since coarser moments and expansions are unused
    int lfar = 0;
    // one-column coupling: workgroups per CU looping over the work items (0: one
    // workgroup per item).  Two gain 1 % on one apply beside the near field (C2: 0.1793
    // against 0.1812 ms) but lose 20 % when several solves share the device (serving,
    // 32 requests on 4 workers: 0.211 against 0.266 solves/s), so the default is 0
    int m2l_persist = 0;
    // once-per-entry near field: both item widths in one launch (C2, beside the coupling:
    // 0.1757 against 0.1797 ms per apply, four runs each; alone it is slower, 76 against
    // 70 us, with the registers of the wider items)
    bool near_one = true;
    // one FP64 column, one degree (<= 8) on every level: the coupling over unordered far
    // pairs, each kernel value used for both clusters of the pair (IGE_M2L_SYM=1).  Off by
    // default: at C2 it halves the kernel evaluations and cuts the VALU instructions per
    // ordered node pair by about a third, yet the kernel is only 7 % faster (86 against
    // 92 us; the values pass through shared memory, the row layout reads the partner's
    // nodes and fields once per row instead of once per three rows, and three workgroups
    // per CU fit instead of four), and the slot reduction costs 4.5 us more: 0.188-0.191
    // against 0.188 ms per apply
    bool m2l_sym = false;
    std::vector<ige::M2LWork> swork;      // row cluster with a chunk of partners of larger index
    ige::DBuf<ige::M2LWork> d_swork;
    ige::DBuf<int32_t> d_spartner, d_sred_ptr, d_sred_idx;   // partners; per cluster its slots
    ige::DBuf<double2> d_spart;           // [items + partners][4][Q] partial couplings
    // many columns: the near-field product on the second stream beside the far field
    // (0: in line after it, 1: from the start, 2: after M2M)
    int batch_overlap = 1;
    bool near_first = false;           // overlap: near field beside the upward pass only, then the coupling alone
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int64_t prof_count = 0;
    int NC = 0;                     // clusters on all levels 0..L
    std::vector<int64_t> lvl_off;   // host copy
    std::vector<ige::M2LWork> work; // M2L work items (targets with chunks of partners)
    std::vector<int32_t> wrk_of_tgt;    // [NC+1] range of work items per target cluster
    std::vector<ige::M2LWork> work1;    // the same for the one-column kernel (its own chunk size)
    std::vector<int32_t> wrk_of_tgt1;
    ige::DBuf<ige::M2LWork> d_work1;
    ige::DBuf<int32_t> d_wrk_of_tgt1;
    // stored coupling blocks (one per unordered far pair)
    bool stored = false;
    bool m2l_generate_one = true;   // single column: evaluate the kernel per apply even when stored
    // shared memory per workgroup of the generated single-column coupling (0: what it
    // needs); more limits its workgroups per CU and leaves registers to the near field
    size_t m2l_lds = 0;
    // wave issue priority of the once-per-entry near-field product (0 or 1, the latter
    // ahead of the coupling kernel's waves on shared SIMDs; measured: no gain per apply,
    // and slower alone, so 0)
    int near_prio = 0;
    // BF16 coupling of wide column chunks: real and imaginary row tiles in one wave
    // (IGE_M2L_RM, default 1)
    bool m2l_rm = true;
    int64_t nfp = 0;

    // device buffers
    ige::DBuf<ige::PatchHdr> d_hdr;
    ige::DBuf<double> d_brk, d_cp;
    ige::DBuf<int32_t> d_dof;
    ige::DBuf<int8_t> d_sgn;
    ige::DBuf<double> d_ext_p, d_ext_q, d_gx, d_gw, d_sx, d_sw;
    ige::DBuf<double> d_eX, d_ePsi, d_ePsiF, d_eC;
    ige::DBuf<int32_t> d_bpair, d_leafdof, d_red_idx;
    ige::DBuf<int8_t> d_leafsgn;
    ige::DBuf<int64_t> d_red_ptr;
    ige::DBuf<double2> d_bval;
    ige::DBuf<double2> d_npart;        // near-field partial results [nslots]
    // near field stored once per distinct entry (product of one column)
    ige::NearCompact cmp;
    bool cmp_on = false;
    int cmp_rs = 2;                      // rows per step of its product (2 or 4)
    ige::NearCmpView cview{};
    ige::DBuf<int32_t> d_cnr, d_cnc, d_cld, d_cidx, d_corder, d_cred_idx, d_cocc_ptr, d_cocc, d_cnp_ptr, d_cnp_leaf, d_cnp_code;
    ige::DBuf<int8_t> d_csym;
    ige::DBuf<int64_t> d_cvoff, d_clst, d_cwpart, d_cred_ptr;
    ige::DBuf<int4> d_cwork;
    ige::DBuf<double2> d_cval, d_cpart;
    ige::DBuf<int64_t> d_lvl_off;
    ige::DBuf<double> d_nodeX, d_nodeT, d_xn, d_T0, d_T1, d_Mp, d_Mq, d_Mdp, d_xnl, d_Rl;
    ige::DBuf<double2> d_sctab;
    ige::DBuf<int32_t> d_inc;
    ige::DBuf<ige::SingularPair> d_sing;
    ige::DBuf<double2> d_sblk;           // singular element-pair blocks (assembly only)
    ige::DBuf<int32_t> d_sing_ptr;
    ige::DBuf<ige::M2LWork> d_work;
    ige::DBuf<int32_t> d_partner;       // source global cluster id per work entry
    ige::DBuf<int32_t> d_wrk_of_tgt;
    ige::DBuf<int> d_err;
    ige::DBuf<int32_t> d_fpair;         // [nfp][2] global cluster ids, t < s
    ige::DBuf<double2> d_G;             // [nfp][Q][Q]
    ige::DBuf<float2> d_G32;            // FP32 copy, made on first use
    ige::DBuf<int64_t> d_fred_ptr;      // [NC+1]
    ige::DBuf<int32_t> d_fred_idx;      // partial slots per cluster, fixed order
    ige::DBuf<double2> d_gpart;         // [2 nfp][4][Q][rb]
    ige::DBuf<double2> d_gtmp;          // [NC][split][4][Q][rb]
    // matrix-core coupling: BF16 blocks (1 plane, or high + low planes), work items of
    // up to 32 partners, block slot per partner entry, operand buffer, partials
    ige::DBuf<__bf16> d_Gb1, d_Gb3, d_vb;
    std::vector<ige::M2LWork> mwork;
    ige::DBuf<ige::M2LWork> d_mwork;
    ige::DBuf<int32_t> d_mpartner, d_gslot, d_mwrk_of_tgt;
    ige::DBuf<float2> d_bmpart;          // matrix-core coupling partials [mwork][4][Q][r]
    ige::DBuf<double> d_Gd, d_vd;       // FP64 matrix-core coupling: blocks, right factors
    ige::DBuf<double2> d_bmpart64;      // FP64 matrix-core coupling partials [mwork][4][Q][r]
    ige::DBuf<double> d_nd, d_xnd;      // FP64 matrix-core near field: ordered-pair blocks, gathered right factors
    ige::DBuf<double2> d_ndpart;        // its partials [near work items][nF][r]
    int nd_fit = -1;                    // those blocks fit in device memory (-1: not yet decided)
    bool near_md_off = false;           // IGE_NEAR_F64=blocks: the unordered-block kernel instead
    int gd_fit = -1;                    // FP64 blocks fit in device memory (-1: not yet decided)
    bool f64mx_off = false;             // FP64 coupling of many columns generated per apply (IGE_M2L_F64=generate)
    ige::DBuf<int32_t> d_morder;         // work items by decreasing partner count (per level with mxl)
    // a degree per level: the matrix-core coupling level by level (levels with far pairs)
    struct MxLevel {
        int lvl = 0, Qr = 0, Qp = 0;     // level, its nodes, padded block size
        int64_t p0 = 0, np = 0;          // its unordered pairs [p0, p0 + np)
        int cl0 = 0, ncl = 0;            // its clusters [cl0, cl0 + ncl)
        int64_t w0 = 0, nw = 0;          // its work items, d_morder[w0, w0 + nw)
        size_t gb_off = 0;               // its blocks in the BF16 store, per plane-block unit
    };
    std::vector<MxLevel> mxl;
    ige::DBuf<int32_t> d_morder_sp;      // work items in cluster order, one contiguous part per XCD (-1: none)
    int64_t n_morder_sp = 0;
    // split-BF16 near-field product (inner solves): blocks per ordered leaf pair,
    // gathered right factors, work items (target leaf, partners), FP32 partials and
    // per-unknown reduction lists
    ige::DBuf<__bf16> d_nb3, d_xnb;
    ige::DBuf<float2> d_nbpart;
    ige::DBuf<ige::M2LWork> d_nbwork;
    ige::DBuf<int32_t> d_nbpartner, d_nbslot, d_nborder, d_nbred_idx;
    ige::DBuf<int64_t> d_nbred_ptr;
    int64_t nb_nwork = 0;
    // apply workspaces (one right-hand side at a time)
    ige::DBuf<double2> d_mom;    // [NC][3][Q]   s^1, s^2, d
    ige::DBuf<double2> d_src;    // [NC][4][Q]   v_x, v_y, v_z, d
    ige::DBuf<double2> d_part;   // [one-column items][4][Q]
    ige::DBuf<double2> d_loc;    // [NC][3][Q]   t^1, t^2, t^d
    ige::DBuf<double2> d_ybuf;   // [leaves][2][rowlen][rowlen] L2P results per leaf
    ige::DBuf<double2> d_x, d_y; // staging for host pointers
    // batched-apply workspaces (r columns, column index innermost)
    int bcap = 0;
    ige::DBuf<double2> d_bnpart;       // near-field partial results [nslots][rb]
    ige::DBuf<double2> d_bnpart_r;     // near-field partial results [nslots][r] (matrix-core product)
    ige::DBuf<double2> d_bmom, d_bsrc, d_bpart, d_bloc, d_bybuf, d_bxt, d_byt, d_bx, d_by;
    // GMRES workspace
    ige::DBuf<double2> d_V, d_w, d_r, d_X, d_F, d_D;
    ige::DBuf<float2> d_V32;           // FP32 Krylov basis of the inner solves of refinement
    ige::DBuf<double2> d_wcur;         // FP64 current basis vectors (with the FP32 basis)
    ige::DBuf<double2> d_h;                          // [2][r][restart + 2] per-pass coefficients
    ige::DBuf<double> d_red, d_scal;
    ige::DBuf<double2> d_gspart, d_gsplit, d_hpack;  // Gram-Schmidt partials, split sums, packed column
    ige::DBuf<double> d_gnp, d_gn;                   // norm partials; [2][r] norms before / after
    ige::DBuf<int> d_grun, d_gflag, d_gact;          // per-column masks
    ige::HBuf<double2> h_hpack;

    ige::DevOp view{};
};

namespace ige {

// autotuned tile choices (ige_op_autotune); absent keys take the built-in default
enum TuneKnob { kTuneM2lNcol = 0, kTuneNearBxNt = 1, kTuneNearMfmaNt = 2, kTuneM2lRb = 3, kTuneM2lDb = 4, kTuneM2lOrder = 5, kTuneM2lF64 = 6, kTuneKnobs = 7 };
inline long long tune_key(int knob, int r, int prec) { return ((long long)knob << 40) | ((long long)r << 8) | prec; }
inline int tune_get(const ige_op_s *op, int knob, int r, int prec, int def)
{
    const auto it = op->tune.find(tune_key(knob, r, prec));
    return it == op->tune.end() ? def : it->second;
}

// stream the apply kernels are launched on (a capture stream while a graph is recorded)
inline hipStream_t lstream(const ige_op_s *op) { return op->lst ? op->lst : op->ctx->stream; }
// whether a profiling event of the given index is recorded at the operator's level
// (level 2 keeps only the boundaries of the block pass, 7-11, and of the coupling kernel, 12-3)
inline bool prof_records(const ige_op_s *op, int i)
{
    return op->profiling == 1 || (op->profiling == 2 && (i == 3 || i == 7 || i == 11 || i == 12));
}

// assembly of geom's operator on ctx's device and stream (throws ige::Status)
ige_op assemble_on(ige_ctx ctx, const ige_geom_s *geom, const ige_params &prm);
// device bytes of an operator planned on the host plus a GMRES with this restart
// device bytes of an operator and an r-column solve with opts (NULL: FP64, no refinement)
size_t planned_device_bytes(const ige_op_s *op, int restart, int r, const ige_solve_opts *opts);

// assembly
void launch_element_data(ige_op op);
void launch_node_geometry(ige_op op);
void launch_near_regular(ige_op op);
int near_regular_sb(int s, int p, int nl);
// doubles of matrix-core operand data per element (see k_element_data)
size_t psi_fragment_doubles(int nl, int G2);
void launch_near_singular(ige_op op);
// values of the once-per-entry near field from the leaf-pair blocks (fixed order)
void launch_near_merge(ige_op op);
// largest rectangle side the once-per-entry product supports
int near_cmp_max();
// its row and column sums into part (one column)
void launch_near_once(ige_op op, const double2 *x, double2 *part, hipStream_t st);
// apply pieces (one right-hand side)
void launch_p2m(ige_op op, const double2 *x);
void launch_m2m(ige_op op);
void launch_m2l(ige_op op, int prec);
// stored coupling blocks: build, FP32 copy, and the M2L + reduce of r columns
// (fields [NC][4][Q][r] in, test-side fields [NC][3][Q][r] out)
void store_coupling(ige_op op);
void ensure_coupling32(ige_op op);
int coupling_rb_max(int Q);
int coupling_split();
void m2l_stored(ige_op op, int r, int prec, const double2 *src, double2 *loc, hipStream_t s);
// one column on the context stream (d_src -> d_gpart, then d_gpart -> d_loc)
void m2l_stored_one(ige_op op, int prec);
void m2l_stored_reduce_one(ige_op op);
int coupling_qp(int Q);   // padded block size of the matrix-core coupling (multiple of 32)
// matrix-core coupling of r columns in BF16 (split 1) or split BF16 (split 3):
// fields [NC][4][Q][r] -> partials per work item [mwork][4][Q][r] (d_bmpart)
void m2l_bf16(ige_op op, int r, int split, const double2 *src, hipStream_t s, hipEvent_t mid = nullptr);
void ensure_coupling_bf16(ige_op op, int split);
// coupling of the FP64 operator on the FP64 matrix cores (many columns): partials d_bmpart64
void ensure_coupling_f64(ige_op op);
void m2l_f64mx(ige_op op, int r, const double2 *src, hipStream_t s, hipEvent_t mid = nullptr);
// whether the FP64 apply of r columns can take (ok) and takes (use) the matrix-core coupling
bool m2l_f64mx_ok(ige_op op, int r);
bool m2l_f64mx_use(ige_op op, int r);
// widest usable coupling chunk (complex columns) for the current staging choice
int m2l_ncol_limit(ige_op op, int r, int split);
// split-BF16 near-field product (yt = near part of A x, [N][r] layout)
void plan_near_bf16(ige_op op, const std::vector<int32_t> &pair, const std::vector<int32_t> &leafdof, int nF);
void ensure_near_bf16(ige_op op, hipStream_t s);
int near_bf16_ok(int nF);
void near_bf16(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s);
// FP64 near field of r >= 56 columns on the FP64 matrix cores (ordered-pair FP64 blocks)
bool near_f64mx_ok(ige_op op, int r);
void near_f64mx(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s);
void launch_m2l_reduce(ige_op op, int prec);
size_t m2l_sym_shared_bytes(int Q);
void launch_l2l(ige_op op);
// near-field product; records mid (if given) between the block pass and the reduction
void launch_spmv(ige_op op, const double2 *x, double2 *y, hipStream_t st, hipEvent_t mid = nullptr);
int near_blk_u(int nF);
int near_mfma_mtw_ok(int nF, int rc);   // the FP64 matrix-core near product supports these blocks   // 64-column groups per block row (template choice)
void launch_l2p_leaf(ige_op op);
void launch_l2p_gather(ige_op op, double2 *y);
// scattered field at npts points (device arrays; src: potential_source_doubles scratch)
size_t potential_source_doubles(ige_op op);
void launch_potential(ige_op op, const double2 *w, int npts, const double *pts, double2 *out, double *src);
// fixed scratch of the allocation-free potential: address lookup (once per device, with
// that device current), the device address (nullptr before the lookup), capacity
void potential_scratch_init(int device);
double *potential_scratch(int device);
size_t potential_scratch_doubles();
// achievable peak of the device on stream s: kind 0 HBM copy (GB/s), 1 BF16 matrix
// cores (TFLOP/s), 2 FP64 matrix cores (TFLOP/s)
double peak_probe(hipStream_t s, int kind);
// raise a kernel's dynamic shared-memory limit above 64 KB once per process
void lds_attr_once(const void *kern, size_t shm);
// scalar single layer right-hand side (kind 0 plane wave of direction a, 1 point source at a)
void launch_rhs_scalar(ige_op op, int kind, const double *a, double2 *f);
void launch_rhs_plane(ige_op op, const double *dir, double2 pol0, double2 pol1, double2 pol2, double2 *f);
// GMRES vector kernels (V: [k][r][n], vectors [r][n]; gate/run/flag: per-column int masks)
struct GsPlan {
    int nchk = 0, nblk = 0;             // entry chunks of the dot and update kernels
    int dot_groups = 1, upd_groups = 1; // basis-index groups per pass (fill the chip at small n r)
};
GsPlan gs_plan(int64_t n, int r, int kmax);
size_t gs_part_count(const GsPlan &g, int r, int kmax);        // double2 partials of a dot pass
size_t gs_split_count(const GsPlan &g, int64_t n, int r);      // double2 split sums of an update
// h[c][kk] = <V[kk][c], w_c> (kk < k, gate columns; 0 elsewhere), nb[c] = |w_c|^2 if nb
void launch_gs_dots(hipStream_t s, const GsPlan &g, int64_t n, int r, const double2 *V, int k, const double2 *w,
                    const int *gate, double2 *part, double2 *h, int hs, double *nb);
// y_c += sign V_c h_c for gate columns; npart (if given) gets per-block |y_c|^2
void launch_gs_update(hipStream_t s, const GsPlan &g, int64_t n, int r, const double2 *V, int k, const double2 *h,
                      int hs, double sign, const int *gate, double2 *y, double2 *split, double *npart);
// the same two passes over an FP32 basis (sums and w, y in FP64)
void launch_gs_dots(hipStream_t s, const GsPlan &g, int64_t n, int r, const float2 *V, int k, const double2 *w,
                    const int *gate, double2 *part, double2 *h, int hs, double *nb);
void launch_gs_update(hipStream_t s, const GsPlan &g, int64_t n, int r, const float2 *V, int k, const double2 *h,
                      int hs, double sign, const int *gate, double2 *y, double2 *split, double *npart);
// nf = |y|^2 of gate columns; scal = 1/|y| for run columns (0 for the others);
// flag (if given) = second Gram-Schmidt pass needed
void launch_gs_norm(hipStream_t s, const GsPlan &g, int r, const double *npart, const int *gate, const int *run,
                    const double *nb, double *nf, double *scal, int *flag);
void launch_gs_pack(hipStream_t s, int r, int k, const double2 *h1, const double2 *h2, int hs, const double *nf,
                    double2 *out);
void launch_axpby(ige_op op, int64_t n, double2 a, const double2 *x, double2 b, double2 *y);
void launch_norm2_b(ige_op op, int r, const double2 *x, double *out);
void launch_scale_cols(ige_op op, int r, const double *s, const double2 *x, double2 *y);
// y_c = s_c x_c and v_c = (FP32) y_c
void launch_scale_cols32(ige_op op, int r, const double *s, const double2 *x, double2 *y, float2 *v);
void launch_axpy_cols(ige_op op, int r, const double *s, const double2 *x, double2 *y);
// x == nullptr: the input is already in xt; y == nullptr: the result stays in yt
void apply_batched(ige_op op, int r, const double2 *x, double2 *y, double2 *xt, double2 *yt, hipEvent_t *ev, int prec);
void batched_to_rows(ige_op op, int r, const double2 *x, double2 *xt, hipStream_t s);
void batched_to_cols(ige_op op, int r, const double2 *yt, double2 *y, hipStream_t s);
void launch_helmholtz_eval(hipStream_t s, int64_t n, double kappa, const double *r2, double2 *out, int prec,
                           const double2 *sctab);

}  // namespace ige
