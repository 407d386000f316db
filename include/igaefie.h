/*
 * igaefie.h -- C ABI of the MI355X (gfx950) isogeometric EFIE library.
 *
 * The library discretises the electric field integral equation
 *     -gamma_t e_i = V_kappa w            (Sec. 2.2, eq. (eq:EFIE))
 * with the div-conforming multipatch spline space S^1 on NURBS patches
 * (Sec. 3.2) and applies the Galerkin matrix of eq. (eq:MSLtested),
 *     A_ij = int int G_k(x-y) phi_j(x).phi_i(y) - k^-2 G_k(x-y) div phi_j div phi_i,
 * G_k(r) = e^{ikr}/(4 pi r) (eq:HelmholtzGreen), compressed by the
 * interpolation-based fast multipole method of Sec. 4.2: exact element-pair
 * quadrature in the near field, tensor Chebyshev interpolation of the localized
 * kernel (eq:lockernel) in the parameter domain for admissible cluster pairs
 * (eq:admissibility, Algorithm 1), with the K_1^(a,b) / K_2 blocks and moment
 * matrices of eq. (eq:FMMlr) and nested cluster bases.  Linear systems are solved
 * with restarted complex GMRES (Sec. 5).
 *
 * Conventions
 *   - every call returns int: IGE_OK (0) or a negative IGE_E* code; the text of the
 *     last error of the calling thread is returned by ige_last_error();
 *   - complex numbers are (re, im) pairs of double (ige_c64), bit-compatible with
 *     C99 double _Complex and torch.complex128;
 *   - a vector of N unknowns uses the canonical unknown order: patch ascending,
 *     then component (0: u-flux, 1: v-flux), then (i2 major, i1 minor); an interface
 *     unknown is numbered where it first occurs and carries sign +1 there and the
 *     sign that makes the normal flux continuous on the other patch;
 *   - r right-hand sides are stored column after column (column c at offset c*N);
 *   - ptr_kind IGE_HOST: pointers are host memory, the call is synchronous;
 *     IGE_DEVICE: pointers are device memory of the context's device and the call is
 *     ordered on the context's stream (it returns before the work completes);
 *   - the caller owns every buffer it passes; the library copies what it keeps.
 *
 * Errors: IGE_EINVAL bad argument / shape / non-conforming geometry;
 *         IGE_ENOMEM device or host allocation failed;
 *         IGE_ENOTCONV GMRES stopped at maxit (x holds the last iterate, stats valid);
 *         IGE_EDEVICE a HIP runtime call failed.
 */
#ifndef IGAEFIE_H
#define IGAEFIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { IGE_OK = 0, IGE_EINVAL = -1, IGE_ENOMEM = -2, IGE_ENOTCONV = -3, IGE_EDEVICE = -4 };
enum { IGE_HOST = 0, IGE_DEVICE = 1 };

typedef struct { double re, im; } ige_c64;

typedef struct ige_ctx_s *ige_ctx;
typedef struct ige_geom_s *ige_geom;
typedef struct ige_op_s *ige_op;

/* Text of the last error raised on the calling thread ("" if none).  Owned by the
 * library; valid until the next call on this thread. */
const char *ige_last_error(void);

/* Library version string. */
const char *ige_version(void);

/* Context: one device and one HIP stream.  device: HIP device ordinal, or -1 for a
 * host-only context that can create geometries and plan operators (ige_op_plan)
 * but not assemble or apply them; it makes no HIP call.
 * hip_stream: a hipStream_t to order all work on, or NULL for a stream the context
 * creates and owns.  One context per host thread.
 * ige_ctx_destroy: IGE_EINVAL while geometries, operators or servers made on the
 * context are not yet destroyed (they use its device and stream). */
int ige_ctx_create(int device, void *hip_stream, ige_ctx *out);
int ige_ctx_destroy(ige_ctx ctx);

/* Geometry: n_patches NURBS maps F_j : [0,1]^2 -> Gamma_j (Sec. 3.1, eq. (def::geom)).
 *   degree [2P]    (p_u, p_v) of each patch, 1..8
 *   n_ctrl [2P]    (n_u, n_v) control points per direction
 *   knots          per patch the open knot vector in u (n_u+p_u+1 values, starting at 0,
 *                  ending at 1, non-decreasing) followed by the one in v; patches
 *                  concatenated
 *   ctrl [sum n_u n_v][4]  control point (x, y, z) and weight w > 0, u index fastest
 * The patches must form a closed, watertight surface whose interfaces coincide as
 * parametrised curves up to orientation (Sec. 3.1), with d_uF x d_vF pointing
 * outwards.  The data are copied; each patch is converted to rational Bezier form
 * per knot span (Bezier extraction, Sec. 5).  IGE_EINVAL on malformed input or an
 * edge without exactly one partner edge. */
int ige_geom_create(ige_ctx ctx, int n_patches, const int *degree, const int *n_ctrl, const double *knots,
                    const double *ctrl, ige_geom *out);
int ige_geom_destroy(ige_geom geom);

/* Discretisation and compression parameters.
 *   p             spline degree of S^1 (Sec. 3.2: S^{p,p-1} x S^{p-1,p}), 1..4
 *   level         m: 2^m x 2^m elements per patch (Sec. 4.1), 0..10
 *   kappa         wavenumber > 0
 *   q             interpolation degree (q+1 Chebyshev nodes per direction), 1..11
 *   eta           admissibility parameter (eq:admissibility); 0 disables the far
 *                 field (dense operator by element quadrature)
 *   gauss_near    g: g x g Gauss points per element for disjoint element pairs (1..8)
 *   gauss_singular gs: Gauss points per variable of the singular sub-rules (1..12)
 *   leaf_depth    d: leaf clusters are 2^d x 2^d elements (leaf level max(0, m-d));
 *                 -1 selects ceil(log2((q+1)/(p+1)))
 *   store_coupling 1: the interpolated kernel matrices G of the admissible blocks
 *                 (Sec. 4.2, the couplings of the H^2 representation) are computed once
 *                 at assembly and stored, one Q x Q complex block per unordered
 *                 cluster pair (G of (s, t) is the transpose of G of (t, s)); every
 *                 apply then streams them (Q^2 * 16 bytes per pair).  0 or -1: G is
 *                 evaluated in every apply (the default: measured faster).
 *   kappa_cap     0: the admissibility condition of the paper (eq:admissibility), which
 *                 does not involve kappa; > 0: a block is admissible only if also
 *                 kappa * max diam <= kappa_cap (coarse clusters many wavelengths
 *                 wide are refined further, so the fixed q keeps its accuracy at high
 *                 kappa; more, smaller far blocks).
 *   kind          IGE_OP_EFIE (0): the EFIE matrix above on S^1;
 *                 IGE_OP_SCALAR (1): the scalar Helmholtz single layer
 *                     A_ij = int int G_k(x-y) phi_j(y) phi_i(x) dsigma dsigma
 *                 on the patchwise tensor B-splines of degree p (Sec. 3.2 with the
 *                 scalar space in place of S^1: (2^m + p)^2 functions per patch, no
 *                 continuity across patches, unknowns ordered patch, i2, i1), compressed
 *                 with the K_2 block alone (eq:FMMlr with the surface elements inside
 *                 the localized kernel).  The scalar operator takes every apply
 *                 precision, refinement and autotuning like the EFIE one; plane-wave
 *                 fields (ige_rhs_plane_wave) and serving refuse it.
 *   q_level       interpolation degree per cluster-tree level l = 0..10 (0: q), 1..15:
 *                 the far blocks of level l are interpolated with q_level[l] + 1 nodes
 *                 per direction (the variable-order form of Sec. 4.2; the paper uses one
 *                 q).  Degrees that grow with kappa * diam of the level's clusters keep
 *                 the accuracy at high kappa without refining the partition; a rule is
 *                 q_l = min(15, max(q, ceil(kappa diam_l / 2) + 5)) on the levels with far
 *                 blocks, with diam_l from ige_op_info of the planned operator.  With
 *                 degrees that differ between levels the generated FP64/FP32 coupling
 *                 takes each level's blocks at their own size in one launch (one and
 *                 many columns), and the matrix-core couplings (BF16, and FP64 of 8 or
 *                 more columns) run one launch per level with that level's padded
 *                 block size.  A degree above 10 on a
 *                 level with far pairs (also one degree q = 11) makes the BF16
 *                 precisions (apply, autotuning, refinement inner solves) refuse with
 *                 IGE_EINVAL; stored coupling blocks need one degree on all levels. */
enum { IGE_OP_EFIE = 0, IGE_OP_SCALAR = 1 };
typedef struct {
    int p, level;
    double kappa;
    int q;
    double eta;
    int gauss_near, gauss_singular, leaf_depth;
    int store_coupling;
    double kappa_cap;
    int kind;
    int q_level[11];
} ige_params;

/* Assemble the operator on the device: element and cluster-node geometry, the
 * near-field Galerkin entries (element-pair quadrature, summed in a fixed order into
 * dense blocks over the leaf function slots of each near leaf pair, glued basis),
 * the far-field partition and the moment and transfer tables.  Synchronous.  The
 * result does not depend on timing: the same inputs give the same bits. */
int ige_op_assemble(ige_geom geom, const ige_params *params, ige_op *out);
int ige_op_destroy(ige_op op);

/* Host-only part of ige_op_assemble: unknowns, cluster and block-cluster trees and
 * the near-field sparsity pattern, without device work (any context).  The result
 * answers ige_op_info / ige_op_dofmap / ige_op_partition; ige_apply, ige_solve and
 * ige_rhs_plane_wave return IGE_EINVAL on it. */
int ige_op_plan(ige_geom geom, const ige_params *params, ige_op *out);

typedef struct {
    int64_t n_dof;          /* N glued unknowns */
    int64_t n_elements;     /* P 4^m */
    int64_t near_nnz;       /* stored near-field entries of the leaf-pair blocks */
    int64_t far_pairs;      /* admissible (ordered) cluster pairs */
    int64_t near_leaf_pairs;
    int64_t singular_pairs; /* element pairs that share a corner */
    int32_t leaf_level, q;
    int64_t device_bytes;   /* device memory held by the operator */
    double assemble_ms;     /* wall time of ige_op_assemble */
    int64_t near_distinct;  /* distinct entries of the symmetric near-field matrix in the
                               glued basis (i <= j): the values the product of one column
                               streams (each once) */
    int32_t q_level[11];    /* interpolation degree of each level 0..leaf_level (0 beyond) */
    double level_diam[11];  /* largest bounding-ball diameter of the clusters of each level
                               0..leaf_level (0 beyond) */
    int32_t m2l_unordered;  /* 1: the one-column FP64 coupling evaluates the kernel once per
                               unordered far pair and serves both clusters (the kernel is
                               symmetric), as asked by IGE_M2L_SYM=1 at creation with one
                               degree (<= 8) on every level; 0: once per ordered pair
                               (default) */
} ige_op_info_t;
int ige_op_info(ige_op op, ige_op_info_t *out);

/* Copy the unknown table to host memory: dof[P][2][n+p][n+p] global index (-1 where
 * the slot is unused) and sgn[P][2][n+p][n+p] (+1/-1), layout [patch][component][i2][i1]. */
int ige_op_dofmap(ige_op op, int32_t *dof, int8_t *sgn);

/* Copy the block-cluster partition to host memory, each list sorted:
 *   far [far_pairs][3]        (level, target cluster, source cluster)
 *   near [near_leaf_pairs][2] (target leaf cluster, source leaf cluster)
 * cluster id on level l: patch*4^l + k2*2^l + k1.  Either pointer may be NULL. */
int ige_op_partition(ige_op op, int32_t *far, int32_t *near);

/* Copy the assembled near-field blocks (the exact Galerkin entries of the
 * non-admissible leaf pairs, Sec. 4.2) to host memory: one dense nF x nF complex
 * block per unordered near leaf pair in the order of ige_op_partition's near list
 * with target <= source, rows over the target leaf's function slots, signs of the
 * glued unknowns folded in, zero rows and columns where a slot holds no unknown.
 * n must equal near_nnz of ige_op_info.  Synchronous.  The assembly sums every entry
 * in a fixed order, so two assemblies of the same operator give the same bits. */
int ige_op_near_blocks(ige_op op, ige_c64 *out, int64_t n);

enum { IGE_F64 = 0, IGE_F32 = 1, IGE_BF16 = 2, IGE_BF16X3 = 3, IGE_BF16X3_ALL = 4 };

/* y = A x for r right-hand sides (A the compressed operator).  x, y: N*r complex.
 * r > 1 runs the batched kernels (columns in chunks, every kernel value and matrix
 * entry read or computed once per chunk); r >= 8 applies the coupling on the FP64
 * matrix cores (see ige_apply_prec, IGE_F64). */
int ige_apply(ige_op op, int r, const ige_c64 *x, ige_c64 *y, int ptr_kind);

/* As ige_apply, with the coupling stage (interpolated-kernel values and their
 * products, M2L) in the given precision:
 *   IGE_F64   FP64 (as ige_apply; with 8 or more columns the kernel matrices are
 *             stored in FP64, both orientations, and applied on the FP64 matrix cores,
 *             unless autotuned otherwise or IGE_M2L_F64=generate);
 *   IGE_F32   FP32 kernel values: evaluated and accumulated in FP32 when generated
 *             on the fly, an FP32 copy of the stored blocks with FP64 accumulation when
 *             stored; relative error about kappa * diam * 2^-23 on the far field;
 *   IGE_BF16  the kernel matrices rounded to BF16 once (stored, both orientations) and
 *             applied with the source fields rounded to BF16 on the BF16 matrix cores
 *             with FP32 accumulation (complex products as one real product);
 *             relative error about 2^-9 on the far field;
 *   IGE_BF16X3 the same with both factors split into a high and a low BF16 part and
 *             three products (high*high + high*low + low*high); about 2^-16;
 *   IGE_BF16X3_ALL  coupling as IGE_BF16X3 and, in addition, the near-field product
 *             from a split-BF16 copy of the FP64-assembled near-field blocks (one block
 *             per ordered leaf pair) with FP32 accumulation; about 2^-16 on the whole
 *             product.  Meant as the inner operator of refined solves.
 * Unless stated, near field, moments and transfers stay FP64.  The FP64 near field of
 * 56 or more columns runs on the FP64 matrix cores from an FP64 copy of the blocks per
 * ordered leaf pair (2 * blocks * Qn * 2Qn * 8 bytes, made on first use when 8 GiB of
 * device memory stay free; IGE_NEAR_F64=blocks keeps the stored blocks and their
 * transposes, as below 56 columns).  The FP32 copy and the
 * BF16 blocks are made on first use (BF16 coupling: 2 * pairs * Qp * 2Qp * 2 bytes per
 * plane, Qp = Q rounded up to 32; split-BF16 near field: 2 * blocks * 2 * Qn * 2Qn * 2
 * bytes, Qn = slots per leaf rounded up to 32). */
int ige_apply_prec(ige_op op, int r, const ige_c64 *x, ige_c64 *y, int ptr_kind, int coupling_prec);

/* Autotuner for the r-column apply in precision prec: times every candidate tile
 * shape of the kernels that apply uses (coordinate descent; each candidate in two
 * rounds of one warm-up and three timed applies on seeded N(0,1) + iN(0,1) columns,
 * HIP events on the context stream, the minimum kept) and keeps a candidate for
 * later applies and solves with the same (r, prec) only when it beats the built-in
 * default by more than 2 %.  Knobs, in choice[] order (-1: not used by this apply
 * or the built-in rule kept, where the rule depends on r):
 *   0 coupling column chunk of the BF16 matrix-core coupling (64, 128, 256 complex
 *     columns, capped where registers would spill),
 *   1 column tiles per wave of the split-BF16 near-field product (1, 2, 4),
 *   2 column tiles per wave of the FP64 matrix-core near-field product of 8 to 55
 *     columns (1, 2, 4),
 *   3 columns per workgroup of the generated FP64/FP32 coupling (1, 2, 4; capped by
 *     shared memory),
 *   4 staging of the BF16 coupling blocks: 1 double-buffered (the next block loaded
 *     step by step during the current product), 0 one buffer with the next block
 *     prefetched into registers,
 *   5 launch order of the BF16 coupling work items: 0 by decreasing partner count,
 *     1 in cluster order with one contiguous part (equal partner counts) per XCD,
 *   6 coupling of the FP64 apply of 8 or more columns: 1 stored FP64 blocks on the
 *     FP64 matrix cores (made on first use, 2 * pairs * Qp * 2Qp * 8 bytes, when that
 *     leaves 8 GiB of device memory free), 0 the kernel evaluated per apply.
 * Returns the number of timed configurations (>= 0) or an error status (< 0). */
int ige_op_autotune(ige_op op, int r, int prec, int *choice, int nchoice);

/* Stage profiling.  ige_op_set_profiling(op, level) creates HIP events (timing only,
 * no system-scope fence) and clears the record; every later apply outside solves
 * records stage boundaries on the streams the stages run on (no host
 * synchronisation): level 1 every boundary, level 2 only those of the block pass and
 * of the coupling kernel (stages 7 and 8 below; the others read 0), for timing the
 * dominant kernels at little cost; level 0 stops recording.  ige_op_stage_times
 * synchronises the streams and returns the average device time (ms) per stage over
 * the last (up to 256) recorded applies: 0 P2M, 1 M2M, 2 M2L, 3 M2L reduce, 4 L2L,
 * 5 near-field product (block pass and reduction), 6 L2P, 7 the block pass alone (the
 * whole near-field product for r > 1), 8 the coupling product alone (stage 2 without
 * the conversion of the source fields to the matrix-core operand layout).  n:
 * capacity of ms[]; returns the stage count (9). */
int ige_op_set_profiling(ige_op op, int on);

/* Scheduling knob: on (default) runs the near-field product on a second stream
 * concurrently with the far-field pipeline; off runs every stage in order on the
 * context stream (used to time each kernel in isolation). */
int ige_op_set_overlap(ige_op op, int on);
int ige_op_stage_times(ige_op op, double *ms, int n);

/* Right-hand side f_i = - int_Gamma e_inc . phi_i dsigma for r plane waves
 * e_inc(x) = pol * exp(i kappa dir.x) (Sec. 3.2, eq. (eq:linsys) with the rotated
 * trace pairing written out): dir [r][3] unit vectors (host), pol [r][3] complex
 * (host), f: N*r complex in ptr_kind memory.  Solving A w = f gives the surface
 * current w with e_s = V~ w (eq:ESLP). */
int ige_rhs_plane_wave(ige_op op, int r, const double *dir, const ige_c64 *pol, ige_c64 *f, int ptr_kind);

/* Right-hand side of the scalar single layer (kind IGE_OP_SCALAR), the Galerkin
 * moments f_i = int_Gamma g phi_i dsigma of r Dirichlet data g (Sec. 2.2: V u = g
 * with the element quadrature of the near field, g x g points per element):
 *   kind IGE_RHS_PLANE: g(x) = exp(i kappa a.x), a a unit direction;
 *   kind IGE_RHS_POINT: g(x) = G_k(x - a), a point source at a (off the surface).
 * a [r][3] (host); f: N*r complex in ptr_kind memory.  IGE_EINVAL on the EFIE
 * operator, a bad kind or non-finite a. */
enum { IGE_RHS_PLANE = 0, IGE_RHS_POINT = 1 };
int ige_rhs_scalar(ige_op op, int r, int kind, const double *a, ige_c64 *f, int ptr_kind);

typedef struct {
    double tol;      /* stop at ||f - A x|| <= tol ||f|| (relative, FP64 operator, x0 as passed) */
    int restart;     /* Krylov basis size before restart (>= 1) */
    int maxit;       /* total iteration cap (inner iterations summed over refinement steps) */
    int refine;      /* 0: GMRES on the FP64 operator; 1: iterative refinement -- FP64
                        residual f - A x, inner GMRES on the inner_prec operator for the
                        correction, x += correction, repeated; each inner solve is at most
                        one GMRES cycle (restart iterations) and stops when its residual
                        estimate is reduced by max(inner_tol, tol / (2 * current relres));
                        a step that reduces the FP64 residual by less than 1/2 while its
                        inner solve claimed twice as much is undone on the columns that
                        got worse and the inner precision moves towards FP64
                        (IGE_BF16X3_ALL or IGE_BF16 -> IGE_BF16X3 -> IGE_F64, and
                        IGE_F32 -> IGE_F64); one right-hand side (r = 1) runs the BF16
                        inner precisions as IGE_F32 (the matrix-core coupling would use
                        one of its 16 columns; the one-column FP32 coupling is faster
                        there and more accurate; IGE_SINGLE_INNER=asked keeps the asked
                        precision); with
                        inner_tol >= 1e-5 the inner solves store their Krylov basis in
                        FP32 (sums, the vector being orthogonalised and the correction
                        in FP64; IGE_INNER_BASIS=fp64 keeps the basis in FP64) */
    double inner_tol;
    int inner_prec;  /* precision of the inner solves (IGE_F64 .. IGE_BF16X3_ALL) */
} ige_solve_opts;

typedef struct {
    int iters;       /* GMRES iterations (all refinement steps) */
    int outer;       /* refinement steps (0 without refinement) */
    double relres;   /* true relative residual ||f - A x|| / ||f|| (FP64 operator) at exit */
    double seconds;  /* wall time of the whole call */
} ige_solve_stats;

/* Solve A x = f with restarted complex GMRES (Sec. 5: no preconditioner), all r
 * right-hand sides at once: every iteration applies the operator to the r current
 * Krylov vectors through the batched kernels; each column keeps its own Krylov
 * basis (classical Gram-Schmidt with one reorthogonalisation, on the device), its
 * own Givens rotations (host) and stops on its own relative residual.
 * x holds the initial guesses on entry.  stats: one entry per right-hand side (may
 * be NULL).  IGE_ENOTCONV if some column stopped at maxit.  Device memory:
 * (restart + 1) * r * N complex for the bases. */
int ige_solve(ige_op op, int r, const ige_c64 *f, ige_c64 *x, int ptr_kind, const ige_solve_opts *opts,
              ige_solve_stats *stats);

/* ---- Serving: scattering solves as they arrive, on one device ----------------
 * A server owns n_workers host threads, each with its own HIP stream on the device
 * of ctx, so the assembly and solve kernels of several requests share the device.
 * A request is one full solve: the operator of geom with the parameters prm
 * (assembled on the worker's stream, Sec. 3-4), the right-hand sides of one or
 * several plane waves e_inc = pol exp(i kappa dir.x) (as ige_rhs_plane_wave), GMRES
 * with opts from x0 = 0 on all of them at once (as ige_solve), and the copy of the
 * solutions to host memory.
 * Admission: requests wait in arrival order and start first-fit when their device
 * footprint (planned on the host at submission: near-field blocks, element and
 * cluster data, Krylov bases of opts.restart vectors per wave, the copies of the
 * blocks that the many-column kernels and the refinement precision make) fits in
 * hbm_budget next to the running requests and the resident operators; the oldest
 * waiting request is overtaken only during its first second of waiting.
 * hbm_budget 0: 80 % of the free device memory.
 * Continuous batching: a worker that takes a request also takes the waiting requests
 * on the same operator (same geom handle and prm) with the same opts, up to
 * max_merge plane waves in all (ige_srv_set_merge, default 64), and solves all their
 * waves as one many-column system (results as for a direct ige_solve of those
 * columns together); a request solved alone gives the same bits as a direct solve.
 * Residency: a worker keeps the assembled operator of its last solve on the device
 * and prefers waiting requests on it (no second assembly); resident operators count
 * in the budget and are freed when a waiting request needs their memory.
 * The caller keeps geom alive until its requests have finished.  Requests that run
 * concurrently share the device and do not synchronise with each other.
 * Timestamps are seconds since the server was created. */
typedef struct ige_srv_s *ige_srv;
typedef struct {
    int state;           /* 0 waiting, 1 running, 2 finished */
    int rc;              /* when finished: IGE_OK, IGE_ENOTCONV (maxit reached), or the error code */
    int iters;           /* GMRES iterations */
    double relres;       /* final true relative residual */
    int64_t n_dof;
    size_t footprint;    /* planned device bytes used for admission */
    double t_submit, t_start, t_done;
    double assemble_s, solve_s;
    int n_waves;         /* plane waves of the request; iters and relres are the largest over them */
    int merged;          /* requests solved together in its solve (1: alone) */
    int reused;          /* 1: ran on an operator already resident on the device */
} ige_srv_stats;
int ige_srv_create(ige_ctx ctx, int n_workers, size_t hbm_budget, ige_srv *out);
/* Queue one request; returns at once with its ticket.  IGE_ENOMEM if its footprint
 * exceeds the budget, IGE_EINVAL on bad parameters. */
int ige_srv_submit(ige_srv srv, ige_geom geom, const ige_params *prm, const double *dir, const ige_c64 *pol,
                   const ige_solve_opts *opts, int64_t *ticket);
/* As ige_srv_submit for n_waves plane waves (1..4096): dir [n_waves][3], pol
 * [n_waves][3] (host, copied), solved together as an n_waves-column system (the
 * many-right-hand-side form of the scattering problem: one operator, several
 * incident directions). */
int ige_srv_submit_waves(ige_srv srv, ige_geom geom, const ige_params *prm, int n_waves, const double *dir,
                         const ige_c64 *pol, const ige_solve_opts *opts, int64_t *ticket);
/* Largest number of plane waves solved together by merging waiting requests on one
 * operator (1: no merging).  Applies to requests submitted afterwards. */
int ige_srv_set_merge(ige_srv srv, int max_waves);
int ige_srv_poll(ige_srv srv, int64_t ticket, ige_srv_stats *stats);   /* non-blocking */
int ige_srv_wait(ige_srv srv, int64_t ticket, ige_srv_stats *stats);   /* blocks until finished */
/* Copy a finished request's solutions (n = n_waves * n_dof complex values, [n_waves][n_dof])
 * to host x. */
int ige_srv_result(ige_srv srv, int64_t ticket, ige_c64 *x, int64_t n);
/* Finish every queued and running request, stop the workers, free everything. */
int ige_srv_destroy(ige_srv srv);

/* Scattered field e_s = V~ w (Sec. 2, eq. (eq:ESLP)) of r densities w [r][N]
 * (ptr_kind memory) at npts points [npts][3] (host) off the surface:
 *   e_s(x) = int G(x-y) w(y) + kappa^-2 grad_x int G(x-y) div w(y) dsigma(y),
 * each element integrated with the g x g Gauss rule of the near field, so points
 * should stay a few element sizes away from the surface.  E: [r][npts][3] complex,
 * host memory.  Synchronous; uses temporary device memory (E * g^2 * 88 bytes).
 * On the scalar single layer (kind IGE_OP_SCALAR) component 0 of each point holds
 * the single layer potential u(x) = int G(x-y) w(y) dsigma(y) and components 1, 2
 * are zero. */
int ige_potential(ige_op op, int r, const ige_c64 *w, int ptr_kind, int npts, const double *points, ige_c64 *E);

/* ige_potential for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels
 * and results, with the per-element source data in a fixed device array of the
 * library (64 MiB per device, held until the process ends) instead of temporary
 * memory.  w [r][N], points [npts][3] and E [r][npts][3] are device memory of the
 * context's device; the call is ordered on the context's stream and returns before
 * the work completes; it calls no hipMalloc/hipFree and makes no host copy (points
 * are not checked for NaN).  IGE_EINVAL if the operator's source data,
 * elements * g^2 * 88 bytes, exceed 64 MiB.  Calls that overlap on one device (two
 * streams, or two host threads) race on that array. */
int ige_potential_noalloc(ige_op op, int r, const ige_c64 *w, int npts, const double *points, ige_c64 *E);

/* Achievable peaks of the context's device, measured by the library's own probe
 * kernels (diagnostic; the benchmarks report roofline fractions against these beside
 * the published figures).  Synchronous; allocates 2 GiB for the copy probe.
 *   IGE_PROBE_HBM:       a grid-stride copy of 1 GiB, *value = GB/s (bytes read + written);
 *   IGE_PROBE_MFMA_BF16: register-only 16x16x32 BF16 matrix-core products (16 independent
 *                        chains per wave, four waves per SIMD on every CU), *value = TFLOP/s;
 *   IGE_PROBE_MFMA_F64:  the same with the 16x16x4 FP64 product (8 chains per wave).
 * Best of 5 timed launches after one warm-up. */
enum { IGE_PROBE_HBM = 0, IGE_PROBE_MFMA_BF16 = 1, IGE_PROBE_MFMA_F64 = 2 };
int ige_peak_probe(ige_ctx ctx, int kind, double *value);

/* Diagnostic: evaluate on the context's device the Helmholtz kernel
 * G_k(r) = e^{ikr}/(4 pi r) (Sec. 2.2, eq. (eq:HelmholtzGreen)) exactly as the
 * coupling stage does in precision prec (IGE_F64: reciprocal square root with one
 * third-order step, table-driven sine and cosine; IGE_F32), from squared distances
 * r2[n] > 0 (host memory) into out[n] (host memory).  Synchronous. */
int ige_helmholtz_eval(ige_ctx ctx, int64_t n, double kappa, const double *r2, ige_c64 *out, int prec);

#ifdef __cplusplus
}
#endif
#endif
