// C ABI of the igaefie library: contexts, geometry, operator assembly, apply,
// right-hand side and GMRES.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <unordered_map>

#include "op.hpp"

namespace {
thread_local std::string g_err;

template <class F>
int guard(F &&f)
{
    try {
        f();
        g_err.clear();
        return IGE_OK;
    } catch (const ige::Status &s) {
        g_err = s.msg;
        return s.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return IGE_ENOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return IGE_EINVAL;
    } catch (...) {
        g_err = "unknown exception";
        return IGE_EINVAL;
    }
}

using ige::DBuf;

// the device of ctx, with the calling thread's last-error state cleared: an error left
// by unrelated code on this thread must not be taken for a failed launch of ours
void set_device(ige_ctx ctx)
{
    IGE_HIP(hipSetDevice(ctx->device));
    (void)hipGetLastError();
}

double2 c2(std::complex<double> z) { return make_double2(z.real(), z.imag()); }
std::complex<double> cz(double2 a) { return {a.x, a.y}; }

// y = A x for one right-hand side; x, y device pointers.
// The near-field product (memory bound) runs on the operator's second stream while
// the far-field pipeline (arithmetic bound) runs on the context stream; the L2P
// gather joins both.  With profiling on, stage boundaries are recorded into one of
// kProfSlots event sets on the stream each stage runs on (no host sync).
// (cos, sin)(j pi/128) / (4 pi), j < 256, rounded from long double: the table of the FP64
// kernel evaluation in the coupling stage
const std::vector<double2> &sincos_table()
{
    static const std::vector<double2> tab = [] {
        std::vector<double2> t(256);
        const long double pi = 3.14159265358979323846264338327950288L, step = pi / 128.0L, f = 0.25L / pi;
        for (int j = 0; j < 256; ++j) t[j] = make_double2((double)(f * cosl(step * j)), (double)(f * sinl(step * j)));
        return t;
    }();
    return tab;
}

void apply_one(ige_op op, const double2 *x, double2 *y, int prec = IGE_F64)
{
    hipStream_t s = ige::lstream(op), s2 = op->aux;
    const bool prof = op->profiling;
    hipEvent_t *ev = prof ? op->prof_ev.data() + (size_t)(op->prof_count % ige_op_s::kProfSlots) * ige_op_s::kProfEv
                          : nullptr;
    auto mark = [&](int i, hipStream_t st) {
        if (prof && ige::prof_records(op, i)) IGE_HIP(hipEventRecord(ev[i], st));
    };
    const bool far = !op->work.empty();
    if (!far || !op->overlap) {
        if (far) {
            mark(0, s);
            ige::launch_p2m(op, x);
            mark(1, s);
            ige::launch_m2m(op);
            mark(2, s);
            mark(12, s);
            ige::launch_m2l(op, prec);
            mark(3, s);
            ige::launch_m2l_reduce(op, prec);
            mark(4, s);
            ige::launch_l2l(op);
            mark(5, s);
            ige::launch_l2p_leaf(op);
            mark(6, s);
        }
        mark(7, s);
        ige::launch_spmv(op, x, y, s, prof ? ev[11] : nullptr);
        mark(8, s);
        if (far) {
            mark(9, s);
            ige::launch_l2p_gather(op, y);
            mark(10, s);
        }
        if (prof) {
            if (!far)
                for (int i : {0, 1, 2, 3, 4, 5, 6, 9, 10, 12}) mark(i, s);
            op->prof_count++;
        }
        return;
    }
    if (op->near_first) {
        // the near-field product beside the short upward pass only; the coupling stage
        // then has the device to itself
        mark(0, s);
        IGE_HIP(hipEventRecord(op->ev_fork, s));
        IGE_HIP(hipStreamWaitEvent(s2, op->ev_fork, 0));
        mark(7, s2);
        ige::launch_spmv(op, x, y, s2, prof ? ev[11] : nullptr);
        mark(8, s2);
        IGE_HIP(hipEventRecord(op->ev_join, s2));
        ige::launch_p2m(op, x);
        mark(1, s);
        ige::launch_m2m(op);
        mark(2, s);
        IGE_HIP(hipStreamWaitEvent(s, op->ev_join, 0));
        mark(12, s);
        ige::launch_m2l(op, prec);
        mark(3, s);
        ige::launch_m2l_reduce(op, prec);
        mark(4, s);
        ige::launch_l2l(op);
        mark(5, s);
        ige::launch_l2p_leaf(op);
        mark(6, s);
        mark(9, s);
        ige::launch_l2p_gather(op, y);
        mark(10, s);
        if (prof) op->prof_count++;
        return;
    }
    // the small upward-pass kernels go first; the near-field product then shares
    // the device with the long coupling stage
    mark(0, s);
    ige::launch_p2m(op, x);
    mark(1, s);
    ige::launch_m2m(op);
    mark(2, s);
    IGE_HIP(hipEventRecord(op->ev_fork, s));
    IGE_HIP(hipStreamWaitEvent(s2, op->ev_fork, 0));
    mark(7, s2);
    ige::launch_spmv(op, x, y, s2, prof ? ev[11] : nullptr);
    mark(8, s2);
    IGE_HIP(hipEventRecord(op->ev_join, s2));
    mark(12, s);
    ige::launch_m2l(op, prec);
    mark(3, s);
    ige::launch_m2l_reduce(op, prec);
    mark(4, s);
    ige::launch_l2l(op);
    mark(5, s);
    ige::launch_l2p_leaf(op);
    mark(6, s);
    IGE_HIP(hipStreamWaitEvent(s, op->ev_join, 0));
    mark(9, s);
    ige::launch_l2p_gather(op, y);
    mark(10, s);
    if (prof) op->prof_count++;
}

void ensure_staging(ige_op op)
{
    if (!op->d_x.p) op->d_x.alloc(op->D.N);
    if (!op->d_y.p) op->d_y.alloc(op->D.N);
}

}  // namespace

namespace ige {
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace ige

extern "C" {

const char *ige_last_error(void) { return g_err.c_str(); }

const char *ige_version(void) { return "igaefie 0.1 (gfx950)"; }

int ige_ctx_create(int device, void *hip_stream, ige_ctx *out)
{
    return guard([&] {
        IGE_REQUIRE(out != nullptr, "out is null");
        if (device == -1) {   // host-only context
            auto *c = new ige_ctx_s();
            c->device = -1;
            *out = c;
            return;
        }
        int cnt = 0;
        IGE_HIP(hipGetDeviceCount(&cnt));
        IGE_REQUIRE(device >= 0 && device < cnt, "device ordinal out of range");
        auto *c = new ige_ctx_s();
        c->device = device;
        try {
            IGE_HIP(hipSetDevice(device));
            ige::potential_scratch_init(device);
            if (hip_stream) {
                c->stream = (hipStream_t)hip_stream;
            } else {
                IGE_HIP(hipStreamCreate(&c->stream));
                c->own_stream = true;
            }
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
    });
}

int ige_ctx_destroy(ige_ctx ctx)
{
    return guard([&] {
        if (!ctx) return;
        IGE_REQUIRE(ctx->users.load() == 0, "the context still has geometries, operators or servers: destroy them first");
        if (ctx->device < 0) {
            delete ctx;
            return;
        }
        if (ctx->own_stream && ctx->stream) {
            (void)hipSetDevice(ctx->device);
            (void)hipStreamDestroy(ctx->stream);
        }
        delete ctx;
    });
}

int ige_geom_create(ige_ctx ctx, int n_patches, const int *degree, const int *n_ctrl, const double *knots,
                    const double *ctrl, ige_geom *out)
{
    return guard([&] {
        IGE_REQUIRE(ctx && out, "null argument");
        auto *g = new ige_geom_s();
        g->ctx = ctx;
        try {
            ige::build_geometry(g->G, n_patches, degree, n_ctrl, knots, ctrl);
        } catch (...) {
            delete g;
            throw;
        }
        ctx->users++;
        *out = g;
    });
}

int ige_geom_destroy(ige_geom geom)
{
    return guard([&] {
        if (!geom) return;
        geom->ctx->users--;
        delete geom;
    });
}

namespace {

void check_params(const ige_params &P)
{
    IGE_REQUIRE(P.p >= 1 && P.p <= ige::kMaxP, "p must be 1..4");
    IGE_REQUIRE(P.level >= 0 && P.level <= 10, "level must be 0..10");
    IGE_REQUIRE(std::isfinite(P.kappa) && P.kappa > 0.0, "kappa must be positive");
    IGE_REQUIRE(P.q >= 1 && P.q <= 11, "q must be 1..11");
    IGE_REQUIRE(std::isfinite(P.eta) && P.eta >= 0.0, "eta must be >= 0");
    IGE_REQUIRE(P.gauss_near >= 1 && P.gauss_near <= ige::kMaxG, "gauss_near must be 1..8");
    IGE_REQUIRE(P.gauss_singular >= 1 && P.gauss_singular <= ige::kMaxGs, "gauss_singular must be 1..12");
    IGE_REQUIRE(P.leaf_depth >= -1 && P.leaf_depth <= 10, "leaf_depth must be -1..10");
    IGE_REQUIRE(P.store_coupling >= -1 && P.store_coupling <= 1, "store_coupling must be -1, 0 or 1");
    IGE_REQUIRE(std::isfinite(P.kappa_cap) && P.kappa_cap >= 0.0, "kappa_cap must be >= 0");
    IGE_REQUIRE(P.kind == IGE_OP_EFIE || P.kind == IGE_OP_SCALAR, "kind must be IGE_OP_EFIE or IGE_OP_SCALAR");
    for (int l = 0; l < 11; ++l)
        IGE_REQUIRE(P.q_level[l] >= 0 && P.q_level[l] <= 15, "q_level entries must be 0 (q) or 1..15");
}

// host part: unknowns, trees, near pattern, singular pairs, far tables
void plan(ige_op op, const ige_geom_s *geom, ige::NearBlocks &A, std::vector<ige::SingularPair> &sing)
{
    const ige_params &P = op->prm;
    int d = P.leaf_depth;
    if (d < 0) d = std::max(0, (int)std::ceil(std::log2((P.q + 1.0) / (P.p + 1.0)) - 1e-12));
    ige::build_discretisation(op->D, geom->G, P.p, P.level, P.kind == IGE_OP_SCALAR ? 1 : 0);
    ige::build_partition(op->T, geom->G, op->D, P.eta, d, P.kappa, P.kappa_cap);
    std::vector<int> ql((size_t)op->T.L + 1);
    for (int l = 0; l <= op->T.L; ++l) ql[l] = P.q_level[l] > 0 ? P.q_level[l] : P.q;
    ige::build_far_tables(op->F, op->D, op->T, ql);
    IGE_REQUIRE(!op->F.varq || P.store_coupling != 1, "stored coupling blocks need one interpolation degree on all levels");
    // row chunks per near-field block (tuning knob IGE_NEAR_CHUNKS, default 2)
    int nch = 2;
    if (const char *e = std::getenv("IGE_NEAR_CHUNKS")) nch = std::max(1, std::min(64, std::atoi(e)));
    ige::build_near_blocks(A, op->D, op->T, nch);
    op->nnz = A.nblk() * A.nF * A.nF;
    // rows per work item of the once-per-entry product (tuning knob IGE_NEAR_ROWS,
    // default 128, at most 128)
    int nrows = 128;
    if (const char *e = std::getenv("IGE_NEAR_ROWS")) nrows = std::max(8, std::min(128, std::atoi(e)));
    ige::build_near_compact(op->cmp, op->D, op->T, A, nrows);
    if (const char *e = std::getenv("IGE_NEAR_RS")) op->cmp_rs = std::atoi(e) == 4 ? 4 : 2;
    if (const char *e = std::getenv("IGE_NEAR_PRIO")) op->near_prio = std::max(0, std::min(1, std::atoi(e)));
    if (const char *e = std::getenv("IGE_M2L_RM")) op->m2l_rm = std::atoi(e) != 0;
    std::vector<double> corners;
    ige::build_singular_pairs(sing, corners, geom->G, op->D, op->T, A);
    op->nsing = (int64_t)sing.size();
    op->lvl_off.assign(op->T.L + 2, 0);
    for (int l = 0; l <= op->T.L; ++l) op->lvl_off[l + 1] = op->lvl_off[l] + ((int64_t)op->D.P << (2 * l));
    op->NC = (int)op->lvl_off[op->T.L + 1];
}

}  // namespace

}  // extern "C"

// device bytes an assembled operator and a single-column GMRES with the given
// restart will hold (estimate from the host plan)
size_t ige::planned_device_bytes(const ige_op_s *op, int restart, int r, const ige_solve_opts *opts)
{
    const ige::Discretisation &D = op->D;
    const int64_t E = (int64_t)D.P * D.n * D.n;
    const int p = D.p, nl = D.scalar ? (p + 1) * (p + 1) : 2 * p * (p + 1), g = op->prm.gauss_near, G2 = g * g;
    const int Q = op->F.Q1 * op->F.Q1;
    const int s = op->T.s, W = s + p, nF = D.scalar ? W * W : 2 * W * (W - 1);
    const int64_t nblk = nF > 0 ? op->nnz / ((int64_t)nF * nF) : 0;
    const size_t R = (size_t)std::max(1, r);
    const size_t nfp = op->T.far.size() / 2, Qp = 32 * (((size_t)Q + 31) / 32), Qn = 32 * (((size_t)nF + 31) / 32);
    size_t b = 0;
    b += (size_t)op->nnz * 16;                                   // near-field blocks
    {   // the near field once per distinct entry, its lists and partial results
        const ige::NearCompact &C = op->cmp;
        b += (size_t)C.nval * 16 + (size_t)C.npart * 16 + C.idx.size() * 4 + C.red_idx.size() * 4 +
             C.red_ptr.size() * 8 + C.occ.size() * 4 + C.wsub.size() * 40;
    }
    b += (size_t)nblk * nF * 3 * 16 * R;                         // partial results (2 row chunks)
    b += (size_t)E * (3 + 4 * nl) * G2 * 8 + (size_t)E * psi_fragment_doubles(nl, G2) * 8 + (size_t)E * 96;
    b += (size_t)op->NC * Q * (9 * 8 + 11 * 16 * R);             // node data, moments, fields
    b += (size_t)op->T.far.size() * 4 * Q * 16 / 4 * R;          // coupling partials (chunks of partners)
    b += (size_t)op->nsing * 24 + (size_t)D.N * 80 * R;
    b += (size_t)op->nsing * nl * nl * 16 + (size_t)nblk * s * s * 4;   // singular pair blocks (assembly)
    b += ((size_t)restart + 1 + 8) * D.N * 16 * R;               // Krylov basis and work vectors
    const ige::GsPlan gp = ige::gs_plan(D.N, (int)R, restart);
    b += (ige::gs_part_count(gp, (int)R, restart) + ige::gs_split_count(gp, D.N, (int)R)) * 16;   // Gram-Schmidt scratch
    // copies made on first use by the many-column kernels
    if (R >= 8) b += nfp * 2 * Qp * 2 * Qp * 8;                  // FP64 coupling blocks
    if (R >= 56) {                                               // ordered-pair FP64 near blocks, operands
        b += (size_t)nblk * 2 * Qn * 2 * Qn * 8;
        const size_t SL = s > 0 ? (size_t)D.n / s : 0;
        b += (size_t)D.P * SL * SL * ((R + 63) / 64) * 64 * 2 * Qn * 8;
    }
    if (opts && opts->refine) {
        const int ip = opts->inner_prec;
        if (opts->inner_tol >= 1e-5) b += ((size_t)restart + 1) * D.N * 8 * R;   // FP32 inner basis
        if (ip == IGE_F32) b += (size_t)op->T.far.size() * Q * Q * 8;           // FP32 coupling values
        if (ip >= IGE_BF16) b += nfp * 2 * (ip == IGE_BF16 ? 1 : 2) * Qp * 2 * Qp * 2;
        if (ip == IGE_BF16X3_ALL) b += (size_t)nblk * 2 * 2 * Qn * 2 * Qn * 2 + (size_t)nblk * nF * 8 * R;
    }
    return b;
}

extern "C" {

int ige_op_plan(ige_geom geom, const ige_params *prm, ige_op *out)
{
    return guard([&] {
        IGE_REQUIRE(geom && prm && out, "null argument");
        check_params(*prm);
        const auto t0 = std::chrono::steady_clock::now();
        auto *op = new ige_op_s();
        op->ctx = geom->ctx;
        op->prm = *prm;
        op->assembled = false;
        try {
            ige::NearBlocks A;
            std::vector<ige::SingularPair> sing;
            plan(op, geom, A, sing);
        } catch (...) {
            delete op;
            throw;
        }
        op->assemble_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        op->ctx->users++;
        *out = op;
    });
}

}  // extern "C"

// assembly of the operator of geom on the device and stream of ctx (throws)
ige_op ige::assemble_on(ige_ctx ctx, const ige_geom_s *geom, const ige_params &prm)
{
    ige_op result = nullptr;
    {
        const ige_params P = prm;
        check_params(P);
        IGE_REQUIRE(ctx->device >= 0, "assembly needs a device context");
        const auto t0 = std::chrono::steady_clock::now();
        set_device(ctx);
        hipStream_t s = ctx->stream;
        auto *op = new ige_op_s();
        op->ctx = ctx;
        op->prm = P;
        try {
            ige::NearBlocks A;
            std::vector<ige::SingularPair> sing;
            plan(op, geom, A, sing);
            op->assembled = true;
            const auto &D = op->D;
            const auto &T = op->T;
            const auto &F = op->F;
            ige::DevOp &v = op->view;
            v.P = D.P; v.p = D.p; v.m = D.m; v.n = D.n; v.nb = D.nb; v.N = D.N;
            v.scalar = D.scalar;
            v.nl = D.scalar ? (D.p + 1) * (D.p + 1) : 2 * D.p * (D.p + 1);
            // factor of the value / divergence term: 1 (scalar), -kappa^-2 (EFIE)
            v.cdiv = D.scalar ? 1.0 : -1.0 / (P.kappa * P.kappa);
            v.L = T.L; v.s = T.s; v.SL = 1 << T.L;
            v.q = F.q; v.Q1 = F.Q1; v.Q = v.Q1 * v.Q1;
            v.varq = F.varq ? 1 : 0;
            for (int l = 0; l < ige::kMaxLev; ++l) v.ql[l] = l <= T.L ? F.ql[l] : F.q;
            v.g = P.gauss_near; v.G2 = v.g * v.g; v.gs = P.gauss_singular;
            v.kappa = P.kappa; v.h = 1.0 / D.n; v.scale_tol = 1e-9 * geom->G.scale;
            v.rowlen = F.rowlen;
            // geometry and tables
            op->d_hdr.upload(geom->G.hdr, s);
            op->d_brk.upload(geom->G.brk, s);
            op->d_cp.upload(geom->G.cp, s);
            v.geo = ige::GeomView{op->d_hdr.p, op->d_brk.p, op->d_cp.p};
            op->d_dof.upload(D.dof, s);
            op->d_sgn.upload(D.sgn, s);
            v.dof = op->d_dof.p; v.sgn = op->d_sgn.p;
            op->d_ext_p.upload(D.ext_p, s);
            op->d_ext_q.upload(D.ext_q, s);
            v.ext_p = op->d_ext_p.p; v.ext_q = op->d_ext_q.p;
            std::vector<double> gx(v.g), gw(v.g), sx(v.gs), sw(v.gs);
            ige::gauss_legendre01(v.g, gx.data(), gw.data());
            ige::gauss_legendre01(v.gs, sx.data(), sw.data());
            op->d_gx.upload(gx, s); op->d_gw.upload(gw, s); op->d_sx.upload(sx, s); op->d_sw.upload(sw, s);
            v.gx = op->d_gx.p; v.gw = op->d_gw.p; v.sx = op->d_sx.p; v.sw = op->d_sw.p;
            std::vector<int32_t> inc((size_t)D.N * 2 * 5);
            for (size_t i = 0; i < D.inc.size(); ++i)
                for (int k = 0; k < 5; ++k) inc[i * 5 + k] = D.inc[i][k];
            op->d_inc.upload(inc, s);
            v.inc = op->d_inc.p;
            op->d_err.alloc(1);
            IGE_HIP(hipMemsetAsync(op->d_err.p, 0, sizeof(int), s));
            v.err = op->d_err.p;
            // a0: element data
            const int64_t E = (int64_t)D.P * D.n * D.n;
            op->d_eX.alloc((size_t)E * 3 * v.G2);
            op->d_ePsi.alloc((size_t)E * 4 * v.nl * v.G2);
            const size_t fragE = ige::psi_fragment_doubles(v.nl, v.G2);
            op->d_ePsiF.alloc((size_t)E * fragE);
            IGE_HIP(hipMemsetAsync(op->d_ePsiF.p, 0, sizeof(double) * E * fragE, s));
            op->d_eC.alloc((size_t)E * 12);
            v.eX = op->d_eX.p; v.ePsi = op->d_ePsi.p; v.ePsiF = op->d_ePsiF.p; v.eC = op->d_eC.p;
            ige::launch_element_data(op);
            // near-field blocks and quadrature
            v.W = A.W; v.nF = A.nF; v.nch = A.nch; v.rc = A.rc; v.nblk = A.nblk();
            op->d_bpair.upload(A.pair, s);
            op->d_leafdof.upload(A.leafdof, s);
            op->d_leafsgn.upload(A.leafsgn, s);
            op->d_red_ptr.upload(A.red_ptr, s);
            op->d_red_idx.upload(A.red_idx, s);
            ige::plan_near_bf16(op, A.pair, A.leafdof, A.nF);
            op->d_bval.alloc(std::max<int64_t>(1, op->nnz));
            IGE_HIP(hipMemsetAsync(op->d_bval.p, 0, sizeof(double2) * op->nnz, s));
            op->d_npart.alloc(std::max<int64_t>(1, A.nslots()));
            v.bpair = op->d_bpair.p; v.bval = op->d_bval.p; v.leafdof = op->d_leafdof.p; v.leafsgn = op->d_leafsgn.p;
            v.red_ptr = op->d_red_ptr.p; v.red_idx = op->d_red_idx.p;
            op->d_sing.upload(sing, s);
            {
                // range of singular pairs per (block, test element of the target leaf):
                // the list is ordered by block, then test element (row major in the leaf)
                const int s2 = T.s * T.s;
                std::vector<int32_t> sptr((size_t)A.nblk() * s2 + 1, 0);
                int64_t prev = -1;
                for (size_t k = 0; k < sing.size(); ++k) {
                    const int64_t e = sing[k].e;
                    const int e1 = (int)(e % D.n), e2 = (int)((e / D.n) % D.n);
                    const int64_t key = (int64_t)sing[k].blk * s2 + (e2 % T.s) * T.s + (e1 % T.s);
                    IGE_REQUIRE(key >= prev, "singular pairs not ordered by block and test element");
                    prev = key;
                    sptr[key + 1]++;
                }
                for (size_t i = 1; i < sptr.size(); ++i) sptr[i] += sptr[i - 1];
                op->d_sing_ptr.upload(sptr, s);
            }
            op->d_sblk.alloc(std::max<size_t>(1, (size_t)op->nsing * v.nl * v.nl));
            v.sing = op->d_sing.p; v.sing_ptr = op->d_sing_ptr.p; v.sblk = op->d_sblk.p;
            // singular element pairs into their own slots, then the regular pairs and those
            // slots summed into the blocks in a fixed order (colour by colour)
            ige::launch_near_singular(op);
            ige::launch_near_regular(op);
            // the same near field once per distinct entry, for the product of one column
            // (IGE_NEAR_COMPACT=0 keeps the leaf-pair blocks for it)
            {
                const ige::NearCompact &C = op->cmp;
                bool on = C.nsub() > 0 && C.maxn <= ige::near_cmp_max();
                if (const char *e = std::getenv("IGE_NEAR_COMPACT")) on = on && std::atoi(e) != 0;
                op->cmp_on = on;
                if (on) {
                    std::vector<int4> wk(C.wsub.size());
                    for (size_t w = 0; w < wk.size(); ++w) wk[w] = make_int4(C.wsub[w], C.wr0[w], C.wr1[w], 0);
                    op->d_cnr.upload(C.nr, s);
                    op->d_cnc.upload(C.nc, s);
                    op->d_cld.upload(C.ld, s);
                    op->d_csym.upload(C.sym, s);
                    op->d_cvoff.upload(C.val, s);
                    op->d_clst.upload(C.lst, s);
                    op->d_cidx.upload(C.idx, s);
                    op->d_cwork.upload(wk, s);
                    op->d_cwpart.upload(C.wpart, s);
                    op->d_corder.upload(C.worder, s);
                    op->d_cred_ptr.upload(C.red_ptr, s);
                    op->d_cred_idx.upload(C.red_idx, s);
                    op->d_cocc_ptr.upload(C.occ_ptr, s);
                    op->d_cocc.upload(C.occ, s);
                    op->d_cnp_ptr.upload(C.np_ptr, s);
                    op->d_cnp_leaf.upload(C.np_leaf, s);
                    op->d_cnp_code.upload(C.np_code, s);
                    op->d_cval.alloc(std::max<int64_t>(1, C.nval));
                    op->d_cpart.alloc(std::max<int64_t>(1, C.npart));
                    ige::NearCmpView &cv = op->cview;
                    cv.nsub = C.nsub();
                    cv.nwork = (int64_t)C.wsub.size();
                    cv.nr = op->d_cnr.p; cv.nc = op->d_cnc.p; cv.ld = op->d_cld.p; cv.sym = op->d_csym.p;
                    cv.val_off = op->d_cvoff.p; cv.lst = op->d_clst.p; cv.idx = op->d_cidx.p;
                    cv.val = op->d_cval.p; cv.work = op->d_cwork.p; cv.wpart = op->d_cwpart.p;
                    cv.order = op->d_corder.p;
                    cv.occ_ptr = op->d_cocc_ptr.p; cv.occ = op->d_cocc.p;
                    cv.np_ptr = op->d_cnp_ptr.p; cv.np_leaf = op->d_cnp_leaf.p; cv.np_code = op->d_cnp_code.p;
                    ige::launch_near_merge(op);
                }
            }
            // cluster tree and far field
            op->d_lvl_off.upload(op->lvl_off, s);
            v.lvl_off = op->d_lvl_off.p;
            op->d_xn.upload(F.xn, s);
            op->d_T0.upload(F.T0, s);
            op->d_T1.upload(F.T1, s);
            op->d_Mp.upload(F.Mp, s);
            op->d_Mq.upload(F.Mq, s);
            op->d_Mdp.upload(F.Mdp, s);
            v.xn = op->d_xn.p; v.T0 = op->d_T0.p; v.T1 = op->d_T1.p;
            op->d_xnl.upload(F.xnl, s);
            op->d_Rl.upload(F.R, s);
            v.xnl = op->d_xnl.p; v.Rl = op->d_Rl.p;
            v.Mp = op->d_Mp.p; v.Mq = op->d_Mq.p; v.Mdp = op->d_Mdp.p;
            op->d_nodeX.alloc((size_t)op->NC * 3 * v.Q);
            op->d_nodeT.alloc((size_t)op->NC * 6 * v.Q);
            // levels of a smaller degree fill only the first (q_l + 1)^2 entries of a field
            IGE_HIP(hipMemsetAsync(op->d_nodeX.p, 0, op->d_nodeX.bytes(), s));
            IGE_HIP(hipMemsetAsync(op->d_nodeT.p, 0, op->d_nodeT.bytes(), s));
            v.nodeX = op->d_nodeX.p; v.nodeT = op->d_nodeT.p;
            op->d_sctab.upload(sincos_table(), s);
            v.sctab = op->d_sctab.p;
            ige::launch_node_geometry(op);
            // M2L work items: partners of each target in chunks
            // partners per M2L work item (tuning knob IGE_M2L_CHUNK, default 8)
            int CH = 8;
            if (const char *e = std::getenv("IGE_M2L_CHUNK")) CH = std::max(1, std::min(64, std::atoi(e)));
            op->overlap = true;
            if (const char *e = std::getenv("IGE_OVERLAP")) op->overlap = std::atoi(e) != 0;
            if (const char *e = std::getenv("IGE_NEAR_FIRST")) op->near_first = std::atoi(e) != 0;
            if (const char *e = std::getenv("IGE_NEAR_ONE")) op->near_one = std::atoi(e) != 0;
            if (const char *e = std::getenv("IGE_BATCH_OVERLAP")) op->batch_overlap = std::max(0, std::min(2, std::atoi(e)));
            if (const char *e = std::getenv("IGE_M2L_PERSIST")) op->m2l_persist = std::max(0, std::min(16, std::atoi(e)));
            op->lfar = T.far.empty() ? T.L + 1 : T.far.front()[0];   // far pairs sorted by level
            // the one-column kernel's items (IGE_M2L_CHUNK1, default 12 partners): longer
            // items leave more of the device to the near-field product beside them (C2:
            // 0.1818-0.1854 ms per apply against 0.1863-0.1885 with 8; alone the coupling
            // kernel takes 98 against 91 us)
            int CH1 = 12;
            if (const char *e = std::getenv("IGE_M2L_CHUNK1")) CH1 = std::max(1, std::min(64, std::atoi(e)));
            std::vector<int32_t> partner;
            for (const auto &f : T.far) partner.push_back((int32_t)(op->lvl_off[f[0]] + f[2]));
            // targets with chunks of up to ch partners, and per target its range of items
            auto chunk_items = [&](int ch, std::vector<ige::M2LWork> &work, std::vector<int32_t> &wot) {
                work.clear();
                wot.assign(op->NC + 1, 0);
                std::vector<int32_t> cnt(op->NC, 0);
                size_t i = 0;
                while (i < T.far.size()) {   // sorted by level, cluster, partner
                    const int lvl = T.far[i][0], tg = T.far[i][1];
                    const int gc = (int)op->lvl_off[lvl] + tg;
                    size_t k = i;
                    while (k < T.far.size() && T.far[k][0] == lvl && T.far[k][1] == tg) ++k;
                    for (size_t b = i; b < k; b += ch) {
                        work.push_back({gc, (int32_t)b, (int32_t)std::min(k, b + ch)});
                        cnt[gc]++;
                    }
                    i = k;
                }
                for (int c = 0; c < op->NC; ++c) wot[c + 1] = wot[c] + cnt[c];
            };
            chunk_items(CH, op->work, op->wrk_of_tgt);
            chunk_items(CH1, op->work1, op->wrk_of_tgt1);
            // unordered far pairs (t < s) and, per cluster, its partial couplings in
            // pair order: slot 2k = row side of pair k (cluster t), 2k+1 = column side (s)
            {
                std::vector<int32_t> fpair;
                for (const auto &f : T.far) {
                    const int32_t gt = (int32_t)(op->lvl_off[f[0]] + f[1]), gs = (int32_t)(op->lvl_off[f[0]] + f[2]);
                    IGE_REQUIRE(gt != gs, "a cluster is admissible with itself");
                    if (gt > gs) continue;
                    IGE_REQUIRE(std::binary_search(T.far.begin(), T.far.end(),
                                                   std::array<int32_t, 3>{f[0], f[2], f[1]}),
                                "far pairs are not symmetric");
                    fpair.push_back(gt);
                    fpair.push_back(gs);
                }
                op->nfp = (int64_t)fpair.size() / 2;
                IGE_REQUIRE(2 * op->nfp == (int64_t)T.far.size(), "far pairs are not symmetric");
                std::vector<int64_t> fptr((size_t)op->NC + 1, 0);
                for (int64_t k = 0; k < op->nfp; ++k) {
                    fptr[fpair[2 * k] + 1]++;
                    fptr[fpair[2 * k + 1] + 1]++;
                }
                for (int c = 0; c < op->NC; ++c) fptr[c + 1] += fptr[c];
                std::vector<int32_t> fidx(fptr[op->NC]);
                std::vector<int64_t> fill(fptr.begin(), fptr.end() - 1);
                for (int64_t k = 0; k < op->nfp; ++k) {
                    fidx[fill[fpair[2 * k]]++] = (int32_t)(2 * k);
                    fidx[fill[fpair[2 * k + 1]]++] = (int32_t)(2 * k + 1);
                }
                // store the blocks only when asked: streaming them was measured slower
                // than evaluating the kernel per apply, at one and at many columns
                op->stored = P.store_coupling == 1 && op->nfp > 0;
                // single column with stored blocks: streamed (default) or evaluated
                // per apply (IGE_M2L_ONE=generate)
                op->m2l_generate_one = false;
                if (const char *e = std::getenv("IGE_M2L_LDS_KB")) op->m2l_lds = (size_t)std::max(0, std::min(150, std::atoi(e))) * 1024;
                if (const char *e = std::getenv("IGE_M2L_ONE")) op->m2l_generate_one = std::string(e) == "generate";
                // many FP64 columns: stored blocks on the FP64 matrix cores (default) or
                // evaluated per apply (IGE_M2L_F64=generate)
                if (const char *e = std::getenv("IGE_M2L_F64")) op->f64mx_off = std::string(e) == "generate";
                // many FP64 columns: near field on ordered-pair FP64 blocks (default) or on
                // the stored unordered blocks and their transposes (IGE_NEAR_F64=blocks)
                if (const char *e = std::getenv("IGE_NEAR_F64")) op->near_md_off = std::string(e) == "blocks";
                if (op->nfp > 0) {
                    op->d_fpair.upload(fpair, s);
                    // matrix-core coupling: per target, work items of up to 32 partners
                    // with the BF16 block slot (2 pair + orientation) of every ordered pair
                    std::unordered_map<int64_t, int32_t> pid;
                    pid.reserve((size_t)op->nfp * 2);
                    for (int64_t k = 0; k < op->nfp; ++k) pid[(int64_t)fpair[2 * k] * op->NC + fpair[2 * k + 1]] = (int32_t)k;
                    std::vector<int32_t> mpart, gslot, mcnt(op->NC, 0);
                    op->mwork.clear();
                    size_t i = 0;
                    while (i < T.far.size()) {
                        const int lvl = T.far[i][0], tg = T.far[i][1];
                        const int32_t gt = (int32_t)(op->lvl_off[lvl] + tg);
                        size_t k = i;
                        const int beg = (int)mpart.size();
                        while (k < T.far.size() && T.far[k][0] == lvl && T.far[k][1] == tg) {
                            const int32_t gs = (int32_t)(op->lvl_off[lvl] + T.far[k][2]);
                            mpart.push_back(gs);
                            gslot.push_back(gt < gs ? 2 * pid.at((int64_t)gt * op->NC + gs)
                                                    : 2 * pid.at((int64_t)gs * op->NC + gt) + 1);
                            ++k;
                        }
                        for (int b = beg; b < (int)mpart.size(); b += 32) {
                            op->mwork.push_back({gt, b, std::min((int)mpart.size(), b + 32)});
                            mcnt[gt]++;
                        }
                        i = k;
                    }
                    std::vector<int32_t> mwt(op->NC + 1, 0);
                    for (int c = 0; c < op->NC; ++c) mwt[c + 1] = mwt[c] + mcnt[c];
                    // launch order: decreasing partner count (long items first)
                    std::vector<int32_t> morder(op->mwork.size());
                    for (size_t w = 0; w < morder.size(); ++w) morder[w] = (int32_t)w;
                    std::stable_sort(morder.begin(), morder.end(), [&](int32_t a, int32_t b) {
                        return op->mwork[a].end - op->mwork[a].beg > op->mwork[b].end - op->mwork[b].beg;
                    });
                    op->d_morder.upload(morder, s);
                    // alternative launch order: the work items in cluster order (neighbouring
                    // targets share partners) cut into 8 contiguous parts of equal partner
                    // counts, part x on XCD x (consecutive workgroups go round-robin over the
                    // eight XCDs), so partners' right factors are reused in that XCD's L2
                    {
                        const size_t nw = op->mwork.size();
                        int64_t total = 0;
                        for (const auto &w : op->mwork) total += w.end - w.beg;
                        std::vector<std::vector<int32_t>> parts(8);
                        int64_t acc = 0;
                        for (size_t w = 0; w < nw; ++w) {
                            const int x = (int)std::min<int64_t>(7, total > 0 ? acc * 8 / total : 0);
                            parts[x].push_back((int32_t)w);
                            acc += op->mwork[w].end - op->mwork[w].beg;
                        }
                        std::vector<int32_t> sp;
                        sp.reserve(nw + 8);
                        size_t longest = 0;
                        for (const auto &pt : parts) longest = std::max(longest, pt.size());
                        for (size_t i = 0; i < longest; ++i)
                            for (int x = 0; x < 8; ++x) sp.push_back(i < parts[x].size() ? parts[x][i] : -1);
                        op->d_morder_sp.upload(sp, s);
                        op->n_morder_sp = (int64_t)sp.size();
                    }
                    if (F.varq) {
                        // a degree per level: the matrix-core coupling runs level by level,
                        // each with its own padded block size; block slots count from the
                        // level's first pair, the launch order sorts within each level
                        op->mxl.clear();
                        for (size_t w = 0; w < morder.size(); ++w) morder[w] = (int32_t)w;
                        int64_t p0 = 0, w0 = 0;
                        size_t goff = 0;
                        while (p0 < op->nfp) {
                            const int32_t g0 = fpair[2 * p0];
                            int lv = 0;
                            while (lv < T.L && g0 >= op->lvl_off[lv + 1]) ++lv;
                            int64_t p1 = p0;
                            while (p1 < op->nfp && fpair[2 * p1] < op->lvl_off[lv + 1]) ++p1;
                            int64_t w1 = w0;
                            while (w1 < (int64_t)op->mwork.size() && op->mwork[w1].tgt < op->lvl_off[lv + 1]) ++w1;
                            ige_op_s::MxLevel L;
                            L.lvl = lv;
                            L.Qr = (F.ql[lv] + 1) * (F.ql[lv] + 1);
                            L.Qp = ige::coupling_qp(L.Qr);
                            L.p0 = p0;
                            L.np = p1 - p0;
                            L.cl0 = (int)op->lvl_off[lv];
                            L.ncl = (int)(op->lvl_off[lv + 1] - op->lvl_off[lv]);
                            L.w0 = w0;
                            L.nw = w1 - w0;
                            L.gb_off = goff;   // in units of Qp x 2Qp blocks of one plane
                            goff += (size_t)L.np * 2 * L.Qp * 2 * L.Qp;
                            for (int64_t w = w0; w < w1; ++w)
                                for (int k = op->mwork[w].beg; k < op->mwork[w].end; ++k) gslot[k] -= (int32_t)(2 * p0);
                            std::stable_sort(morder.begin() + w0, morder.begin() + w1, [&](int32_t a, int32_t b) {
                                return op->mwork[a].end - op->mwork[a].beg > op->mwork[b].end - op->mwork[b].beg;
                            });
                            op->mxl.push_back(L);
                            p0 = p1;
                            w0 = w1;
                        }
                        IGE_REQUIRE(w0 == (int64_t)op->mwork.size(), "coupling work items are not grouped by level");
                        op->d_morder.upload(morder, s);
                    }
                    op->d_mwork.upload(op->mwork, s);
                    op->d_mpartner.upload(mpart, s);
                    op->d_gslot.upload(gslot, s);
                    op->d_mwrk_of_tgt.upload(mwt, s);
                }
                if (op->stored) {
                    const int rbm = ige::coupling_rb_max(v.Q);
                    op->d_fred_ptr.upload(fptr, s);
                    op->d_fred_idx.upload(fidx, s);
                    op->d_gpart.alloc((size_t)2 * op->nfp * 4 * v.Q * rbm);
                    op->d_gtmp.alloc((size_t)op->NC * ige::coupling_split() * 4 * v.Q * rbm);
                }
                if (op->stored) op->d_G.alloc((size_t)op->nfp * v.Q * v.Q);
            }
            op->d_work.upload(op->work, s);
            op->d_partner.upload(partner, s);
            op->d_wrk_of_tgt.upload(op->wrk_of_tgt, s);
            op->d_work1.upload(op->work1, s);
            op->d_wrk_of_tgt1.upload(op->wrk_of_tgt1, s);
            op->d_mom.alloc((size_t)op->NC * 3 * v.Q);
            op->d_src.alloc((size_t)op->NC * 4 * v.Q);
            // source fields of the levels above the coarsest far level are never written
            // (the upward pass stops there) but the matrix-core coupling stages them
            IGE_HIP(hipMemsetAsync(op->d_src.p, 0, op->d_src.bytes(), s));
            op->d_loc.alloc((size_t)op->NC * 3 * v.Q);
            op->d_ybuf.alloc((size_t)D.P * v.SL * v.SL * 2 * F.rowlen * F.rowlen);
            op->d_part.alloc(std::max<size_t>(1, op->work1.size()) * 4 * v.Q);
            // one FP64 column, one degree (<= 8) on every level: the coupling over unordered
            // pairs when asked (IGE_M2L_SYM=1), items = cluster t with up to
            // IGE_M2L_SYM_CHUNK (default 4) partners s > t
            op->m2l_sym = false;
            if (const char *e = std::getenv("IGE_M2L_SYM"))
                op->m2l_sym = std::atoi(e) != 0 && !F.varq && !T.far.empty() && v.Q <= 81 &&
                              ige::m2l_sym_shared_bytes(v.Q) <= (size_t)64 * 1024;
            if (op->m2l_sym) {
                int CHS = 4;
                if (const char *e = std::getenv("IGE_M2L_SYM_CHUNK")) CHS = std::max(1, std::min(64, std::atoi(e)));
                std::vector<int32_t> spart;
                op->swork.clear();
                size_t i = 0;
                while (i < T.far.size()) {   // sorted by level, cluster, partner
                    const int lvl = T.far[i][0], tg = T.far[i][1];
                    const int beg = (int)spart.size();
                    size_t k = i;
                    for (; k < T.far.size() && T.far[k][0] == lvl && T.far[k][1] == tg; ++k)
                        if (T.far[k][2] > tg) spart.push_back((int32_t)(op->lvl_off[lvl] + T.far[k][2]));
                    for (int b = beg; b < (int)spart.size(); b += CHS)
                        op->swork.push_back({(int32_t)(op->lvl_off[lvl] + tg), b, std::min((int)spart.size(), b + CHS)});
                    i = k;
                }
                IGE_REQUIRE(2 * spart.size() == T.far.size(), "far pairs are not symmetric");
                // the longest items launch first
                std::stable_sort(op->swork.begin(), op->swork.end(), [](const ige::M2LWork &a, const ige::M2LWork &b) {
                    return a.end - a.beg > b.end - b.beg;
                });
                // per cluster its slots: the row sides of its items, then the column sides
                // of its pairs, in that fixed order
                const int nw = (int)op->swork.size();
                std::vector<int32_t> sptr((size_t)op->NC + 1, 0);
                for (const auto &w : op->swork) sptr[w.tgt + 1]++;
                for (int32_t c : spart) sptr[c + 1]++;
                for (int c = 0; c < op->NC; ++c) sptr[c + 1] += sptr[c];
                std::vector<int32_t> sidx(sptr[op->NC]), fill(sptr.begin(), sptr.end() - 1);
                for (int w = 0; w < nw; ++w) sidx[fill[op->swork[w].tgt]++] = w;
                for (size_t k = 0; k < spart.size(); ++k) sidx[fill[spart[k]]++] = nw + (int32_t)k;
                op->d_swork.upload(op->swork, s);
                op->d_spartner.upload(spart, s);
                op->d_sred_ptr.upload(sptr, s);
                op->d_sred_idx.upload(sidx, s);
                op->d_spart.alloc(((size_t)nw + spart.size()) * 4 * v.Q);
            }
            if (op->stored) ige::store_coupling(op);
            IGE_HIP(hipStreamCreate(&op->aux));
            // fork/join between two streams of one device: no system-scope fence (the
            // kernels' own releases and acquires order the device memory; 5 us per apply)
            IGE_HIP(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming | hipEventDisableSystemFence));
            IGE_HIP(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming | hipEventDisableSystemFence));
            IGE_HIP(hipStreamSynchronize(s));
            int err = 0;
            IGE_HIP(hipMemcpy(&err, op->d_err.p, sizeof(int), hipMemcpyDeviceToHost));
            IGE_REQUIRE(err == 0, "near-field assembly produced entries outside the leaf function slots");
            op->d_sblk.release();
            v.sblk = nullptr;
        } catch (...) {
            delete op;
            throw;
        }
        op->assemble_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        ctx->users++;
        result = op;
    }
    return result;
}

extern "C" {

int ige_op_assemble(ige_geom geom, const ige_params *prm, ige_op *out)
{
    return guard([&] {
        IGE_REQUIRE(geom && prm && out, "null argument");
        *out = ige::assemble_on(geom->ctx, geom, *prm);
    });
}

int ige_op_destroy(ige_op op)
{
    return guard([&] {
        if (!op) return;
        op->ctx->users--;
        if (!op->assembled) {
            delete op;
            return;
        }
        (void)hipSetDevice(op->ctx->device);
        (void)hipStreamSynchronize(op->ctx->stream);
        for (auto &e : op->prof_ev)
            if (e) (void)hipEventDestroy(e);
        if (op->aux) {
            (void)hipStreamSynchronize(op->aux);
            (void)hipStreamDestroy(op->aux);
        }
        if (op->gstream) (void)hipStreamDestroy(op->gstream);
        if (op->ev_fork) (void)hipEventDestroy(op->ev_fork);
        if (op->ev_join) (void)hipEventDestroy(op->ev_join);
        delete op;
    });
}

int ige_op_info(ige_op op, ige_op_info_t *out)
{
    return guard([&] {
        IGE_REQUIRE(op && out, "null argument");
        ige_op_info_t r{};
        r.n_dof = op->D.N;
        r.n_elements = (int64_t)op->D.P * op->D.n * op->D.n;
        r.near_nnz = op->nnz;
        r.near_distinct = op->cmp.distinct;
        r.m2l_unordered = op->m2l_sym ? 1 : 0;
        r.far_pairs = (int64_t)op->T.far.size();
        r.near_leaf_pairs = (int64_t)op->T.near.size();
        r.singular_pairs = op->nsing;
        r.leaf_level = op->T.L;
        r.q = op->F.q;
        for (int l = 0; l <= op->T.L && l < 11; ++l) {
            r.q_level[l] = op->F.ql[l];
            r.level_diam[l] = op->T.diam[l];
        }
        size_t b = 0;
        b += op->d_hdr.bytes() + op->d_brk.bytes() + op->d_cp.bytes() + op->d_dof.bytes() + op->d_sgn.bytes();
        b += op->d_ext_p.bytes() + op->d_ext_q.bytes() + op->d_eX.bytes() + op->d_ePsi.bytes() + op->d_eC.bytes();
        b += op->d_ePsiF.bytes() + op->d_bpair.bytes() + op->d_leafdof.bytes() + op->d_leafsgn.bytes();
        b += op->d_red_ptr.bytes() + op->d_red_idx.bytes() + op->d_bval.bytes() + op->d_npart.bytes() + op->d_bnpart.bytes();
        b += op->d_nodeX.bytes() + op->d_nodeT.bytes() + op->d_G.bytes() + op->d_G32.bytes() + op->d_gpart.bytes() + op->d_gtmp.bytes();
        b += op->d_fpair.bytes() + op->d_fred_ptr.bytes() + op->d_fred_idx.bytes();
        b += op->d_Gb1.bytes() + op->d_Gb3.bytes() + op->d_vb.bytes() + op->d_bmpart.bytes();
        b += op->d_Gd.bytes() + op->d_vd.bytes() + op->d_bmpart64.bytes();
        b += op->d_nd.bytes() + op->d_xnd.bytes() + op->d_ndpart.bytes();
        b += op->d_nb3.bytes() + op->d_xnb.bytes() + op->d_nbpart.bytes() + op->d_nbwork.bytes();
        b += op->d_nbpartner.bytes() + op->d_nbslot.bytes() + op->d_nborder.bytes() + op->d_nbred_ptr.bytes();
        b += op->d_nbred_idx.bytes() + op->d_morder.bytes();
        b += op->d_Mp.bytes() * 3 + op->d_inc.bytes() + op->d_sing.bytes() + op->d_work.bytes();
        b += op->d_work1.bytes() + op->d_wrk_of_tgt1.bytes() + op->d_wrk_of_tgt.bytes();
        b += op->d_partner.bytes() + op->d_mom.bytes() + op->d_src.bytes() + op->d_loc.bytes() + op->d_part.bytes();
        b += op->d_swork.bytes() + op->d_spartner.bytes() + op->d_sred_ptr.bytes() + op->d_sred_idx.bytes() + op->d_spart.bytes();
        b += op->d_x.bytes() + op->d_y.bytes() + op->d_V.bytes() + op->d_w.bytes() + op->d_r.bytes();
        b += op->d_cnr.bytes() + op->d_cnc.bytes() + op->d_cld.bytes() + op->d_cidx.bytes() + op->d_corder.bytes() + op->d_cred_idx.bytes();
        b += op->d_cocc_ptr.bytes() + op->d_cocc.bytes() + op->d_cnp_ptr.bytes() + op->d_cnp_leaf.bytes();
        b += op->d_cnp_code.bytes() + op->d_csym.bytes() + op->d_cvoff.bytes() + op->d_clst.bytes();
        b += op->d_cwpart.bytes() + op->d_cred_ptr.bytes() + op->d_cwork.bytes() + op->d_cval.bytes() + op->d_cpart.bytes();
        r.device_bytes = (int64_t)b;
        r.assemble_ms = op->assemble_ms;
        *out = r;
    });
}

int ige_op_dofmap(ige_op op, int32_t *dof, int8_t *sgn)
{
    return guard([&] {
        IGE_REQUIRE(op, "null operator");
        if (dof) std::memcpy(dof, op->D.dof.data(), sizeof(int32_t) * op->D.dof.size());
        if (sgn) std::memcpy(sgn, op->D.sgn.data(), op->D.sgn.size());
    });
}

int ige_op_partition(ige_op op, int32_t *far, int32_t *near)
{
    return guard([&] {
        IGE_REQUIRE(op, "null operator");
        if (far)
            for (size_t i = 0; i < op->T.far.size(); ++i)
                for (int k = 0; k < 3; ++k) far[3 * i + k] = op->T.far[i][k];
        if (near)
            for (size_t i = 0; i < op->T.near.size(); ++i)
                for (int k = 0; k < 2; ++k) near[2 * i + k] = op->T.near[i][k];
    });
}

int ige_op_near_blocks(ige_op op, ige_c64 *out, int64_t n)
{
    return guard([&] {
        IGE_REQUIRE(op && out, "null argument");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        IGE_REQUIRE(n == op->nnz, "n must equal near_nnz");
        set_device(op->ctx);
        IGE_HIP(hipStreamSynchronize(op->ctx->stream));
        if (n > 0) IGE_HIP(hipMemcpy(out, op->d_bval.p, sizeof(double2) * (size_t)n, hipMemcpyDeviceToHost));
    });
}

int ige_op_set_profiling(ige_op op, int on)
{
    return guard([&] {
        IGE_REQUIRE(op, "null operator");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        set_device(op->ctx);
        if (on && op->prof_ev.empty()) {
            op->prof_ev.assign((size_t)ige_op_s::kProfSlots * ige_op_s::kProfEv, nullptr);
            // timing only: no system-scope fence at each record (a fence writes back and
            // invalidates the caches; the streams are synchronised before the read-out)
            for (auto &e : op->prof_ev) IGE_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        }
        IGE_REQUIRE(on >= 0 && on <= 2, "profiling level must be 0, 1 or 2");
        op->profiling = on;
        if (on) op->prof_level_rec = on;
        op->prof_count = 0;
    });
}

int ige_op_set_overlap(ige_op op, int on)
{
    return guard([&] {
        IGE_REQUIRE(op, "null operator");
        op->overlap = on != 0;
    });
}

int ige_op_stage_times(ige_op op, double *ms, int n)
{
    int cnt = 0;
    int rc = guard([&] {
        IGE_REQUIRE(op && ms, "null argument");
        const int nst = 9;
        for (int i = 0; i < std::min(n, nst); ++i) ms[i] = 0.0;
        const int64_t k = std::min<int64_t>(op->prof_count, ige_op_s::kProfSlots);
        if (k > 0) {
            set_device(op->ctx);
            IGE_HIP(hipStreamSynchronize(op->ctx->stream));
            IGE_HIP(hipStreamSynchronize(op->aux));
            // stage -> (begin event, end event); L2P = leaf part + gather part
            const int pairs[9][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {7, 8}, {5, 6}, {7, 11}, {12, 3}};
            for (int64_t sl = 0; sl < k; ++sl) {
                hipEvent_t *ev = op->prof_ev.data() + sl * ige_op_s::kProfEv;
                for (int i = 0; i < std::min(n, nst); ++i) {
                    if (op->prof_level_rec == 2 && i != 7 && i != 8) continue;   // not recorded
                    float t = 0.f;
                    IGE_HIP(hipEventElapsedTime(&t, ev[pairs[i][0]], ev[pairs[i][1]]));
                    double v = t;
                    if (i == 6) {
                        float t2 = 0.f;
                        IGE_HIP(hipEventElapsedTime(&t2, ev[9], ev[10]));
                        v += t2;
                    }
                    ms[i] += v / (double)k;
                }
            }
        }
        cnt = nst;
    });
    return rc == IGE_OK ? cnt : rc;
}

namespace {
// batched workspaces for r columns
void ensure_batched(ige_op op, int r)
{
    if (op->bcap >= r) return;
    const ige::DevOp &v = op->view;
    const size_t Q = v.Q;
    op->d_bmom.alloc((size_t)op->NC * 3 * Q * r);
    op->d_bsrc.alloc((size_t)op->NC * 4 * Q * r);
    IGE_HIP(hipMemsetAsync(op->d_bsrc.p, 0, op->d_bsrc.bytes(), op->ctx->stream));   // as d_src
    op->d_bloc.alloc((size_t)op->NC * 3 * Q * r);
    op->d_bpart.alloc(std::max<size_t>(1, op->work.size()) * 4 * Q * r);
    op->d_bybuf.alloc((size_t)v.P * v.SL * v.SL * 2 * v.rowlen * v.rowlen * r);
    op->d_bxt.alloc((size_t)v.N * r);
    op->d_bnpart.alloc(std::max<size_t>(1, (size_t)v.nblk * v.nF * (1 + v.nch)) * 4);
    op->d_byt.alloc((size_t)v.N * r);
    op->bcap = r;
}
}  // namespace

namespace {
// A captured HIP graph of the operator body (every kernel of one apply between the
// copy of x into the op's own input buffer and the copy of the result out of its
// output buffer) for one column count and precision.  The first apply with a new
// (r, prec) runs eagerly (it sizes every buffer and makes the one-time BF16 copies),
// the second is captured, later ones replay it: one launch instead of one per kernel.
// Valid while the op's buffers keep their size, i.e. within one solve.
struct ApplyGraph {
    int r = -1, prec = -1, eager = 0;
    hipGraphExec_t exec = nullptr;
    hipStream_t launched = nullptr;   // stream of the last launch of exec
    // an executable graph is destroyed only after its launches have completed (also when
    // a solve unwinds from an error with a launch still in flight)
    void reset()
    {
        if (exec) {
            if (launched) (void)hipStreamSynchronize(launched);
            (void)hipGraphExecDestroy(exec);
        }
        exec = nullptr;
        launched = nullptr;
        eager = 0;
    }
    ~ApplyGraph() { reset(); }
};

bool graphs_enabled()
{
    const char *e = std::getenv("IGE_GRAPH");
    return !e || std::string(e) != "0";
}

void run_graph(ige_op op, ApplyGraph *g, int r, int prec, const std::function<void()> &body)
{
    hipStream_t s = op->ctx->stream;
    if (g->exec && g->r == r && g->prec == prec) {
        g->launched = s;
        IGE_HIP(hipGraphLaunch(g->exec, s));
        return;
    }
    if (g->r != r || g->prec != prec) {
        g->reset();
        g->r = r;
        g->prec = prec;
    }
    if (g->eager == 0) {
        g->eager = 1;
        body();
        return;
    }
    if (!op->gstream) IGE_HIP(hipStreamCreateWithFlags(&op->gstream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    IGE_HIP(hipStreamBeginCapture(op->gstream, hipStreamCaptureModeThreadLocal));
    op->lst = op->gstream;
    try {
        body();
    } catch (...) {
        op->lst = nullptr;
        (void)hipStreamEndCapture(op->gstream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    op->lst = nullptr;
    IGE_HIP(hipStreamEndCapture(op->gstream, &graph));
    const hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    IGE_HIP(e);
    g->launched = s;
    IGE_HIP(hipGraphLaunch(g->exec, s));
}

// the matrix-core couplings take blocks of at most 128 padded nodes (degree at most 10
// on every level with far pairs; with a degree per level, one launch per level).
// Other operators couple on the generated FP64/FP32 kernels
bool mx_coupling_ok(const ige_op_s *op)
{
    if (!op->F.varq) return op->F.q <= 10;
    for (const auto &L : op->mxl)
        if (L.Qp > 128) return false;
    return true;
}

// y = A x for r device columns ([r][N]) in the given precision; with g, the operator
// body runs as a captured graph (not while profiling)
void apply_dev(ige_op op, int r, const double2 *x, double2 *y, int prec, ApplyGraph *g = nullptr)
{
    const bool graph = g && !op->profiling && graphs_enabled();
    hipStream_t s = op->ctx->stream;
    const int64_t N = op->D.N;
    if (r == 1 && prec <= IGE_F32) {
        for (int c = 0; c < r; ++c) {
            const double2 *xc = x + (size_t)c * N;
            double2 *yc = y + (size_t)c * N;
            if (!graph) {
                apply_one(op, xc, yc, prec);
                continue;
            }
            ensure_staging(op);
            IGE_HIP(hipMemcpyAsync(op->d_x.p, xc, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
            run_graph(op, g, 1, prec, [&] { apply_one(op, op->d_x.p, op->d_y.p, prec); });
            IGE_HIP(hipMemcpyAsync(yc, op->d_y.p, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
        }
        return;
    }
    ensure_batched(op, r);
    if (!graph) {
        hipEvent_t *ev = op->profiling
                             ? op->prof_ev.data() + (size_t)(op->prof_count % ige_op_s::kProfSlots) * ige_op_s::kProfEv
                             : nullptr;
        ige::apply_batched(op, r, x, y, op->d_bxt.p, op->d_byt.p, ev, prec);
        if (ev) op->prof_count++;
        return;
    }
    ige::batched_to_rows(op, r, x, op->d_bxt.p, s);
    run_graph(op, g, r, prec,
              [&] { ige::apply_batched(op, r, nullptr, nullptr, op->d_bxt.p, op->d_byt.p, nullptr, prec); });
    ige::batched_to_cols(op, r, op->d_byt.p, y, s);
}

int apply_impl(ige_op op, int r, const ige_c64 *x, ige_c64 *y, int ptr_kind, int prec)
{
    return guard([&] {
        IGE_REQUIRE(op && x && y && r >= 1, "bad apply arguments");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        IGE_REQUIRE(ptr_kind == IGE_HOST || ptr_kind == IGE_DEVICE, "bad ptr_kind");
        IGE_REQUIRE(prec >= IGE_F64 && prec <= IGE_BF16X3_ALL, "bad coupling precision");
        IGE_REQUIRE(prec <= IGE_F32 || mx_coupling_ok(op),
                    "the BF16 couplings need interpolation degrees of at most 10 on the levels with far pairs");
        set_device(op->ctx);
        const int64_t N = op->D.N;
        hipStream_t s = op->ctx->stream;
        if (ptr_kind == IGE_DEVICE) {
            apply_dev(op, r, reinterpret_cast<const double2 *>(x), reinterpret_cast<double2 *>(y), prec);
            return;
        }
        if (op->d_bx.n < (size_t)N * r) {
            op->d_bx.alloc((size_t)N * r);
            op->d_by.alloc((size_t)N * r);
        }
        IGE_HIP(hipMemcpyAsync(op->d_bx.p, x, sizeof(double2) * N * r, hipMemcpyHostToDevice, s));
        apply_dev(op, r, op->d_bx.p, op->d_by.p, prec);
        IGE_HIP(hipMemcpyAsync(y, op->d_by.p, sizeof(double2) * N * r, hipMemcpyDeviceToHost, s));
        IGE_HIP(hipStreamSynchronize(s));
    });
}
}  // namespace

int ige_apply(ige_op op, int r, const ige_c64 *x, ige_c64 *y, int ptr_kind)
{
    return apply_impl(op, r, x, y, ptr_kind, IGE_F64);
}

int ige_apply_prec(ige_op op, int r, const ige_c64 *x, ige_c64 *y, int ptr_kind, int coupling_prec)
{
    return apply_impl(op, r, x, y, ptr_kind, coupling_prec);
}

int ige_op_autotune(ige_op op, int r, int prec, int *choice, int nchoice)
{
    int tried = 0;
    int rc = guard([&] {
        IGE_REQUIRE(op && r >= 1 && (choice || nchoice == 0), "bad autotune arguments");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        IGE_REQUIRE(prec >= IGE_F64 && prec <= IGE_BF16X3_ALL, "bad precision");
        IGE_REQUIRE(prec <= IGE_F32 || mx_coupling_ok(op),
                    "the BF16 couplings need interpolation degrees of at most 10 on the levels with far pairs");
        set_device(op->ctx);
        const int64_t N = op->D.N;
        hipStream_t s = op->ctx->stream;
        // seeded N(0,1) + i N(0,1) input columns
        std::vector<double2> xh((size_t)r * N);
        uint64_t st = 0x9e3779b97f4a7c15ull;
        auto unif = [&] {
            st ^= st << 13;
            st ^= st >> 7;
            st ^= st << 17;
            return ((st >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        };
        for (auto &v : xh) {
            const double a = std::sqrt(-2.0 * std::log(unif())), t = 6.283185307179586 * unif();
            v = make_double2(a * std::cos(t), a * std::sin(t));
        }
        ige::DBuf<double2> dx, dy;
        dx.upload(xh, s);
        dy.alloc(xh.size());
        hipEvent_t e0, e1;
        IGE_HIP(hipEventCreate(&e0));
        IGE_HIP(hipEventCreate(&e1));
        auto time_apply = [&] {
            apply_dev(op, r, dx.p, dy.p, prec);   // warm-up (sizes buffers for this choice)
            IGE_HIP(hipEventRecord(e0, s));
            for (int i = 0; i < 3; ++i) apply_dev(op, r, dx.p, dy.p, prec);
            IGE_HIP(hipEventRecord(e1, s));
            IGE_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            IGE_HIP(hipEventElapsedTime(&ms, e0, e1));
            ++tried;
            return ms / 3.0;
        };
        // the default choice of a knob (what the launchers take without a tuned value)
        auto default_of = [&](int id) {
            switch (id) {
                case ige::kTuneM2lDb: return 1;
                case ige::kTuneM2lOrder: return 0;
                case ige::kTuneM2lF64: return 1;
                case ige::kTuneM2lNcol: return -1;   // the smallest chunk holding all columns
                case ige::kTuneNearBxNt: return r > 32 ? 4 : (r > 16 ? 2 : 1);
                case ige::kTuneNearMfmaNt: return r > 16 ? 2 : 1;
                default: return -1;                   // the largest that fits
            }
        };
        // coordinate descent over the knobs that the (r, prec) apply uses
        const bool mx = r > 1 && prec >= IGE_BF16 && op->mxl.empty(), near_bx = r > 1 && prec == IGE_BF16X3_ALL;
        const bool near_mfma = r >= 8 && prec != IGE_BF16X3_ALL && ige::near_mfma_mtw_ok(op->view.nF, op->view.rc) &&
                               !ige::near_f64mx_ok(op, r);
        // FP64 coupling on the matrix cores (default) against the generated kernel, whose
        // columns per workgroup are tuned only where it is the default
        const bool f64mx = prec == IGE_F64 && ige::m2l_f64mx_ok(op, r);
        const bool gen = r > 1 && prec <= IGE_F32 && !op->stored && !op->work.empty() && !f64mx;
        const int split = prec == IGE_BF16 ? 1 : 3;
        struct Knob {
            bool on;
            int id, key_prec;
            std::vector<int> cand;
        };
        const bool mxon = mx && !op->mwork.empty();
        const Knob knobs[ige::kTuneKnobs] = {{mxon, ige::kTuneM2lOrder, split, {1}},
                                            {mxon, ige::kTuneM2lDb, split, {1, 0}},
                                            {mxon, ige::kTuneM2lNcol, split, {64, 128, 256}},
                                            {near_bx, ige::kTuneNearBxNt, 0, {1, 2, 4}},
                                            {near_mfma, ige::kTuneNearMfmaNt, 0, {1, 2, 4}},
                                            {gen, ige::kTuneM2lRb, prec, {1, 2, 4}},
                                            {f64mx, ige::kTuneM2lF64, IGE_F64, {0}}};
        // each candidate timed in two rounds (minimum kept); a candidate replaces the
        // default only when it is more than 2 % faster (the timings vary by about that)
        std::vector<int> chosen(ige::kTuneKnobs, -1);
        for (const Knob &k : knobs) {
            if (!k.on) continue;
            const long long key = ige::tune_key(k.id, r, k.key_prec);
            op->tune.erase(key);
            std::vector<double> best(k.cand.size() + 1, 1e300);   // last slot: the default
            for (int round = 0; round < 2; ++round) {
                op->tune.erase(key);
                best.back() = std::min(best.back(), time_apply());
                for (size_t c = 0; c < k.cand.size(); ++c) {
                    const int v = k.cand[c];
                    if (k.id == ige::kTuneM2lNcol && v > ige::m2l_ncol_limit(op, r, split)) continue;   // not usable
                    op->tune[key] = v;
                    best[c] = std::min(best[c], time_apply());
                }
            }
            size_t bi = k.cand.size();
            for (size_t c = 0; c < k.cand.size(); ++c)
                if (best[c] < 0.98 * best[bi]) bi = c;
            if (bi == k.cand.size()) {
                op->tune.erase(key);
                chosen[k.id] = default_of(k.id);
            } else {
                op->tune[key] = k.cand[bi];
                chosen[k.id] = k.cand[bi];
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        IGE_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < std::min(nchoice, (int)ige::kTuneKnobs); ++i) choice[i] = chosen[i];
    });
    return rc == IGE_OK ? tried : rc;
}

int ige_rhs_scalar(ige_op op, int r, int kind, const double *a, ige_c64 *f, int ptr_kind)
{
    return guard([&] {
        IGE_REQUIRE(op && a && f && r >= 1, "bad rhs arguments");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        IGE_REQUIRE(op->view.scalar, "the operator is not the scalar single layer");
        IGE_REQUIRE(kind == IGE_RHS_PLANE || kind == IGE_RHS_POINT, "kind must be IGE_RHS_PLANE or IGE_RHS_POINT");
        IGE_REQUIRE(ptr_kind == IGE_HOST || ptr_kind == IGE_DEVICE, "bad ptr_kind");
        set_device(op->ctx);
        const int64_t N = op->D.N;
        hipStream_t s = op->ctx->stream;
        if (ptr_kind == IGE_HOST) ensure_staging(op);
        for (int c = 0; c < r; ++c) {
            const double *ac = a + 3 * c;
            IGE_REQUIRE(std::isfinite(ac[0]) && std::isfinite(ac[1]) && std::isfinite(ac[2]), "a must be finite");
            double2 *fc = reinterpret_cast<double2 *>(f) + (size_t)c * N;
            double2 *dst = (ptr_kind == IGE_HOST) ? op->d_y.p : fc;
            ige::launch_rhs_scalar(op, kind, ac, dst);
            if (ptr_kind == IGE_HOST) {
                IGE_HIP(hipMemcpyAsync(fc, op->d_y.p, sizeof(double2) * N, hipMemcpyDeviceToHost, s));
                IGE_HIP(hipStreamSynchronize(s));
            }
        }
    });
}

int ige_rhs_plane_wave(ige_op op, int r, const double *dir, const ige_c64 *pol, ige_c64 *f, int ptr_kind)
{
    return guard([&] {
        IGE_REQUIRE(op && dir && pol && f && r >= 1, "bad rhs arguments");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        IGE_REQUIRE(!op->view.scalar, "the operator is the scalar single layer: use ige_rhs_scalar");
        IGE_REQUIRE(ptr_kind == IGE_HOST || ptr_kind == IGE_DEVICE, "bad ptr_kind");
        set_device(op->ctx);
        const int64_t N = op->D.N;
        hipStream_t s = op->ctx->stream;
        if (ptr_kind == IGE_HOST) ensure_staging(op);
        for (int c = 0; c < r; ++c) {
            const double *d = dir + 3 * c;
            IGE_REQUIRE(std::isfinite(d[0]) && std::isfinite(d[1]) && std::isfinite(d[2]), "direction must be finite");
            const ige_c64 *pc = pol + 3 * c;
            double2 *fc = reinterpret_cast<double2 *>(f) + (size_t)c * N;
            double2 *dst = (ptr_kind == IGE_HOST) ? op->d_y.p : fc;
            ige::launch_rhs_plane(op, d, make_double2(pc[0].re, pc[0].im), make_double2(pc[1].re, pc[1].im),
                                  make_double2(pc[2].re, pc[2].im), dst);
            if (ptr_kind == IGE_HOST) {
                IGE_HIP(hipMemcpyAsync(fc, op->d_y.p, sizeof(double2) * N, hipMemcpyDeviceToHost, s));
                IGE_HIP(hipStreamSynchronize(s));
            }
        }
    });
}

namespace {
using Cx = std::complex<double>;

struct GmresOut {
    std::vector<int> iters;
    std::vector<double> relres_est;
};

// Restarted GMRES for the r columns of B (device, [r][N]) on the operator in
// precision prec, starting from X (device, [r][N], updated in place); each column
// stops when its residual estimate reaches tol * ||B_c||.  it_cap: per-column
// iteration budget.
// progress lines on stderr (one per GMRES cycle and refinement step) with IGE_SOLVE_LOG=1
bool solve_log()
{
    static const bool on = [] {
        const char *e = std::getenv("IGE_SOLVE_LOG");
        return e && std::atoi(e) != 0;
    }();
    return on;
}

// b32: the Krylov basis stored in FP32 (inner solves of refinement); the vector being
// orthogonalised, every sum and the solution stay FP64, and the operator is applied to
// the FP64 basis vector before rounding
void gmres_batched(ige_op op, int r, const double2 *B, double2 *X, const std::vector<double> &tol, int m,
                   const std::vector<int> &it_cap,
                   int prec, GmresOut &out, bool b32 = false, ApplyGraph *gkeep = nullptr)
{
    const int64_t N = op->D.N;
    hipStream_t s = op->ctx->stream;
    const size_t need = (size_t)(m + 1) * r * N;
    if (b32) {
        if (op->d_V32.n < need) op->d_V32.alloc(need);
        if (op->d_wcur.n < (size_t)r * N) op->d_wcur.alloc((size_t)r * N);
    } else if (op->d_V.n < need) {
        op->d_V.alloc(need);
    }
    if (op->d_w.n < (size_t)r * N) op->d_w.alloc((size_t)r * N);
    const int hs = m + 2;
    const ige::GsPlan gp = ige::gs_plan(N, r, m);
    auto grow = [](auto &buf, size_t n) {
        if (buf.n < n) buf.alloc(n);
    };
    grow(op->d_h, (size_t)2 * r * hs);
    grow(op->d_red, (size_t)r);
    grow(op->d_scal, (size_t)r);
    grow(op->d_gspart, ige::gs_part_count(gp, r, m));
    grow(op->d_gsplit, std::max<size_t>(1, ige::gs_split_count(gp, N, r)));
    grow(op->d_hpack, (size_t)r * (m + 1));
    grow(op->d_gnp, (size_t)r * gp.nblk);
    grow(op->d_gn, (size_t)2 * r);
    grow(op->d_grun, (size_t)r);
    grow(op->d_gflag, (size_t)r);
    grow(op->d_gact, (size_t)r);
    op->h_hpack.ensure((size_t)r * (m + 1));
    double2 *split = ige::gs_split_count(gp, N, r) ? op->d_gsplit.p : nullptr;
    double2 *h1 = op->d_h.p, *h2 = op->d_h.p + (size_t)r * hs;
    double *nb = op->d_gn.p, *nf = op->d_gn.p + r;
    double2 *V = b32 ? nullptr : op->d_V.p, *W = op->d_w.p;
    float2 *V32 = b32 ? op->d_V32.p : nullptr;
    auto dots = [&](int k, const double2 *w, const int *gate, double2 *h, double *nbp) {
        if (b32) ige::launch_gs_dots(s, gp, N, r, V32, k, w, gate, op->d_gspart.p, h, hs, nbp);
        else ige::launch_gs_dots(s, gp, N, r, V, k, w, gate, op->d_gspart.p, h, hs, nbp);
    };
    auto update = [&](int k, const double2 *h, double sign, const int *gate, double2 *y, double *np) {
        if (b32) ige::launch_gs_update(s, gp, N, r, V32, k, h, hs, sign, gate, y, split, np);
        else ige::launch_gs_update(s, gp, N, r, V, k, h, hs, sign, gate, y, split, np);
    };
    // basis vector j scaled in place (x = y), with its FP32 copy in the FP32 basis
    auto scale_basis = [&](int j, double2 *x) {
        if (b32) ige::launch_scale_cols32(op, r, op->d_scal.p, x, x, V32 + (size_t)j * r * N);
        else ige::launch_scale_cols(op, r, op->d_scal.p, x, x);
    };
    auto norms = [&](const double2 *v) {
        std::vector<double> h(r);
        ige::launch_norm2_b(op, r, v, op->d_red.p);
        IGE_HIP(hipMemcpyAsync(h.data(), op->d_red.p, sizeof(double) * r, hipMemcpyDeviceToHost, s));
        IGE_HIP(hipStreamSynchronize(s));
        return h;
    };
    auto upload_mask = [&](const std::vector<char> &mk, int *dst) {
        std::vector<int> v(mk.begin(), mk.end());
        IGE_HIP(hipMemcpyAsync(dst, v.data(), sizeof(int) * r, hipMemcpyHostToDevice, s));
        IGE_HIP(hipStreamSynchronize(s));   // v leaves scope
    };
    // the apply graph (captured once, replayed): the caller's when given, so that the
    // inner solves of successive refinement steps reuse one graph
    ApplyGraph local;
    ApplyGraph &ag = gkeep ? *gkeep : local;
    const std::vector<double> bnorm = norms(B);
    out.iters.assign(r, 0);
    out.relres_est.assign(r, 0.0);
    std::vector<std::vector<Cx>> H(r, std::vector<Cx>((size_t)(m + 1) * m)), cs(r, std::vector<Cx>(m)),
        sn(r, std::vector<Cx>(m)), g(r, std::vector<Cx>(m + 1));
    while (true) {
        bool budget = false;
        for (int c = 0; c < r; ++c) budget = budget || out.iters[c] < it_cap[c];
        if (!budget) return;   // every column used its iterations
        // V0 = B - A X (FP64; with the FP32 basis in the current-vector buffer)
        apply_dev(op, r, X, W, prec, &ag);
        double2 *cur = b32 ? op->d_wcur.p : V, *nxt = W;
        ige::launch_axpby(op, (int64_t)r * N, make_double2(1, 0), B, make_double2(0, 0), cur);
        ige::launch_axpby(op, (int64_t)r * N, make_double2(-1, 0), W, make_double2(1, 0), cur);
        std::vector<double> beta = norms(cur);
        std::vector<char> act(r);
        int nact = 0;
        for (int c = 0; c < r; ++c) {
            out.relres_est[c] = bnorm[c] > 0 ? beta[c] / bnorm[c] : 0.0;
            act[c] = bnorm[c] > 0 && out.relres_est[c] > tol[c] && out.iters[c] < it_cap[c];
            nact += act[c];
        }
        if (solve_log()) {
            double worst = 0.0;
            int itmax = 0;
            for (int c = 0; c < r; ++c) {
                worst = std::max(worst, out.relres_est[c]);
                itmax = std::max(itmax, out.iters[c]);
            }
            std::fprintf(stderr, "[igaefie] gmres cycle: %d of %d columns active, iterations %d, max relres %.3e\n",
                         nact, r, itmax, worst);
            std::fflush(stderr);
        }
        if (nact == 0) return;
        std::vector<double> sc(r);
        for (int c = 0; c < r; ++c) sc[c] = act[c] ? 1.0 / beta[c] : 0.0;
        IGE_HIP(hipMemcpyAsync(op->d_scal.p, sc.data(), sizeof(double) * r, hipMemcpyHostToDevice, s));
        scale_basis(0, cur);
        IGE_HIP(hipStreamSynchronize(s));   // sc leaves scope
        std::vector<int> jdone(r, 0);
        for (int c = 0; c < r; ++c) {
            std::fill(g[c].begin(), g[c].end(), Cx(0));
            g[c][0] = beta[c];
        }
        std::vector<char> run = act;
        upload_mask(run, op->d_grun.p);
        for (int jj = 0; jj < m; ++jj) {
            double2 *Vj = b32 ? cur : V + (size_t)jj * r * N, *Vj1 = b32 ? nxt : V + (size_t)(jj + 1) * r * N;
            apply_dev(op, r, Vj, Vj1, prec, &ag);
            // Gram-Schmidt pass 1 on the running columns, pass 2 where it lost more than half
            dots(jj + 1, Vj1, op->d_grun.p, h1, nb);
            update(jj + 1, h1, -1.0, op->d_grun.p, Vj1, op->d_gnp.p);
            ige::launch_gs_norm(s, gp, r, op->d_gnp.p, op->d_grun.p, op->d_grun.p, nb, nf, op->d_scal.p,
                                op->d_gflag.p);
            dots(jj + 1, Vj1, op->d_gflag.p, h2, nullptr);
            update(jj + 1, h2, -1.0, op->d_gflag.p, Vj1, op->d_gnp.p);
            ige::launch_gs_norm(s, gp, r, op->d_gnp.p, op->d_gflag.p, op->d_grun.p, nullptr, nf, op->d_scal.p,
                                nullptr);
            scale_basis(jj + 1, Vj1);
            if (b32) std::swap(cur, nxt);
            ige::launch_gs_pack(s, r, jj + 1, h1, h2, hs, nf, op->d_hpack.p);
            const double2 *hp = op->h_hpack.p;
            IGE_HIP(hipMemcpyAsync(op->h_hpack.p, op->d_hpack.p, sizeof(double2) * r * (jj + 2), hipMemcpyDeviceToHost,
                                   s));
            IGE_HIP(hipStreamSynchronize(s));
            int nrun = 0;
            bool changed = false;
            std::vector<Cx> hc(jj + 2);
            for (int c = 0; c < r; ++c) {
                if (!run[c]) continue;
                for (int i = 0; i <= jj + 1; ++i) hc[i] = cz(hp[(size_t)c * (jj + 2) + i]);
                const double hn = hc[jj + 1].real();
                for (int i = 0; i < jj; ++i) {   // rotations [[conj c, conj s], [-s, c]]
                    const Cx t = std::conj(cs[c][i]) * hc[i] + std::conj(sn[c][i]) * hc[i + 1];
                    hc[i + 1] = -sn[c][i] * hc[i] + cs[c][i] * hc[i + 1];
                    hc[i] = t;
                }
                const double rho = std::sqrt(std::norm(hc[jj]) + std::norm(hc[jj + 1]));
                cs[c][jj] = rho > 0 ? hc[jj] / rho : Cx(1);
                sn[c][jj] = rho > 0 ? hc[jj + 1] / rho : Cx(0);
                hc[jj] = rho;
                g[c][jj + 1] = -sn[c][jj] * g[c][jj];
                g[c][jj] = std::conj(cs[c][jj]) * g[c][jj];
                for (int i = 0; i <= jj; ++i) H[c][(size_t)i * m + jj] = hc[i];
                out.iters[c]++;
                jdone[c] = jj + 1;
                out.relres_est[c] = std::abs(g[c][jj + 1]) / bnorm[c];
                if (out.relres_est[c] <= tol[c] || out.iters[c] >= it_cap[c] || hn == 0.0) {
                    run[c] = 0;
                    changed = true;
                }
                nrun += run[c];
            }
            if (solve_log() && (jj + 1) % 250 == 0) {   // progress inside long cycles
                double worst = 0.0;
                for (int c = 0; c < r; ++c)
                    if (run[c]) worst = std::max(worst, out.relres_est[c]);
                std::fprintf(stderr, "[igaefie] gmres: %d iterations into the cycle, %d columns running, max relres %.3e\n",
                             jj + 1, nrun, worst);
                std::fflush(stderr);
            }
            if (nrun == 0) break;
            if (changed) upload_mask(run, op->d_grun.p);
        }
        // X_c += V_c y_c with y_c = H_c^-1 g_c (upper triangular)
        int kmax = 0;
        for (int c = 0; c < r; ++c) kmax = std::max(kmax, jdone[c]);
        std::vector<double2> ny((size_t)r * hs, make_double2(0, 0));
        for (int c = 0; c < r; ++c) {
            const int k = jdone[c];
            std::vector<Cx> yv(k);
            for (int i = k - 1; i >= 0; --i) {
                Cx acc = g[c][i];
                for (int t = i + 1; t < k; ++t) acc -= H[c][(size_t)i * m + t] * yv[t];
                yv[i] = acc / H[c][(size_t)i * m + i];
            }
            for (int i = 0; i < k; ++i) ny[(size_t)c * hs + i] = c2(yv[i]);
        }
        IGE_HIP(hipMemcpyAsync(op->d_h.p, ny.data(), sizeof(double2) * r * hs, hipMemcpyHostToDevice, s));
        std::vector<char> upd(r);
        for (int c = 0; c < r; ++c) upd[c] = jdone[c] > 0;
        upload_mask(upd, op->d_gact.p);
        if (kmax > 0) update(kmax, op->d_h.p, 1.0, op->d_gact.p, X, nullptr);
    }
}
}  // namespace

int ige_solve(ige_op op, int r, const ige_c64 *f, ige_c64 *x, int ptr_kind, const ige_solve_opts *opts,
              ige_solve_stats *stats)
{
    bool notconv = false;
    int rc = guard([&] {
        IGE_REQUIRE(op && f && x && opts && r >= 1, "bad solve arguments");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        IGE_REQUIRE(ptr_kind == IGE_HOST || ptr_kind == IGE_DEVICE, "bad ptr_kind");
        IGE_REQUIRE(opts->restart >= 1 && opts->maxit >= 0 && std::isfinite(opts->tol) && opts->tol >= 0.0,
                    "bad solve options");
        IGE_REQUIRE(!opts->refine || (opts->inner_prec >= IGE_F64 && opts->inner_prec <= IGE_BF16X3_ALL),
                    "bad inner precision");
        IGE_REQUIRE(!opts->refine || (std::isfinite(opts->inner_tol) && opts->inner_tol > 0.0 && opts->inner_tol < 1.0),
                    "inner_tol must be in (0, 1)");
        IGE_REQUIRE(!opts->refine || opts->inner_prec <= IGE_F32 || mx_coupling_ok(op),
                    "the BF16 couplings need interpolation degrees of at most 10 on the levels with far pairs");
        set_device(op->ctx);
        const auto t0 = std::chrono::steady_clock::now();
        const int64_t N = op->D.N;
        hipStream_t s = op->ctx->stream;
        const double2 *F;
        double2 *X;
        if (ptr_kind == IGE_HOST) {
            if (op->d_F.n < (size_t)r * N) {
                op->d_F.alloc((size_t)r * N);
                op->d_X.alloc((size_t)r * N);
            }
            IGE_HIP(hipMemcpyAsync(op->d_F.p, f, sizeof(double2) * r * N, hipMemcpyHostToDevice, s));
            IGE_HIP(hipMemcpyAsync(op->d_X.p, x, sizeof(double2) * r * N, hipMemcpyHostToDevice, s));
            F = op->d_F.p;
            X = op->d_X.p;
        } else {
            F = reinterpret_cast<const double2 *>(f);
            X = reinterpret_cast<double2 *>(x);
        }
        std::vector<int> iters(r, 0), outer(r, 0);
        std::vector<double> relres(r, 0.0);
        GmresOut go;
        if (!opts->refine) {
            gmres_batched(op, r, F, X, std::vector<double>(r, opts->tol), opts->restart, std::vector<int>(r, opts->maxit),
                          IGE_F64, go);
            iters = go.iters;
        } else {
            // iterative refinement: FP64 residual, low-precision inner correction
            if (op->d_r.n < (size_t)r * N) op->d_r.alloc((size_t)r * N);
            if (op->d_D.n < (size_t)r * N) op->d_D.alloc((size_t)r * N);
            if (op->d_red.n < (size_t)r) op->d_red.alloc(r);
            std::vector<double> fn(r);
            ige::launch_norm2_b(op, r, F, op->d_red.p);
            IGE_HIP(hipMemcpyAsync(fn.data(), op->d_red.p, sizeof(double) * r, hipMemcpyDeviceToHost, s));
            IGE_HIP(hipStreamSynchronize(s));
            // each inner solve is one GMRES cycle at most: the restart is an outer step with
            // the true FP64 residual, so a cycle never continues past the point where the
            // inner operator's rounding stops the true inner residual from decreasing
            ApplyGraph ag64, ag_inner;
            // inner precision in use; a refinement step whose FP64 residual contracts by
            // less than 1/2 while the inner solve claimed at least twice as much is limited
            // by the inner operator's error: its growing columns are undone and the inner
            // precision moves one rung towards FP64 (split near field -> split coupling -> FP64)
            int cur = opts->inner_prec;
            // one right-hand side: the BF16 matrix-core couplings would fill one of their 16
            // columns and the near field would take the leaf-pair blocks; the FP32 coupling
            // on the one-column kernels is faster there and at least as accurate (C2 size:
            // 0.27 against 0.67 s per solve; IGE_SINGLE_INNER=asked keeps the asked precision)
            const char *esi = std::getenv("IGE_SINGLE_INNER");
            if (r == 1 && cur >= IGE_BF16 && !(esi && std::string(esi) == "asked")) cur = IGE_F32;
            // inner solves keep their Krylov basis in FP32 when they stop at a relative
            // residual of 1e-5 or more (FP32 rounding of the basis, 6e-8, stays far below);
            // IGE_INNER_BASIS=fp64 keeps it in FP64
            const char *eb = std::getenv("IGE_INNER_BASIS");
            const bool inner_b32 = (!eb || std::string(eb) != "fp64") && opts->inner_tol >= 1e-5;
            std::vector<double> prev(r, 0.0), est(r, 0.0), undo(r, 0.0);
            std::vector<int> lastcap(r, 0);
            for (int step = 0; step <= opts->maxit; ++step) {
                apply_dev(op, r, X, op->d_r.p, IGE_F64, &ag64);
                ige::launch_axpby(op, (int64_t)r * N, make_double2(1, 0), F, make_double2(-1, 0), op->d_r.p);
                std::vector<double> rn(r);
                ige::launch_norm2_b(op, r, op->d_r.p, op->d_red.p);
                IGE_HIP(hipMemcpyAsync(rn.data(), op->d_red.p, sizeof(double) * r, hipMemcpyDeviceToHost, s));
                IGE_HIP(hipStreamSynchronize(s));
                if (cur != IGE_F64) {
                    bool bad = false, back = false;
                    for (int c = 0; c < r; ++c) {
                        undo[c] = 0.0;
                        if (lastcap[c] == 0 || prev[c] <= 0.0) continue;
                        const double ratio = (fn[c] > 0 ? rn[c] / fn[c] : 0.0) / prev[c];
                        if (ratio > 0.5 && ratio > 2.0 * est[c]) {
                            bad = true;
                            if (ratio > 1.0) {
                                undo[c] = -1.0;
                                back = true;
                            }
                        }
                    }
                    std::fill(lastcap.begin(), lastcap.end(), 0);
                    if (bad) {
                        cur = cur == IGE_BF16X3_ALL || cur == IGE_BF16 ? IGE_BF16X3 : IGE_F64;
                        if (back) {   // x_c -= correction_c on the columns that got worse
                            IGE_HIP(hipMemcpyAsync(op->d_scal.p, undo.data(), sizeof(double) * r, hipMemcpyHostToDevice, s));
                            ige::launch_axpy_cols(op, r, op->d_scal.p, op->d_D.p, X);
                            IGE_HIP(hipStreamSynchronize(s));
                            continue;   // recompute the residual of the restored columns
                        }
                    }
                }
                bool any = false;
                std::vector<int> cap(r);
                std::vector<double> itol(r);
                for (int c = 0; c < r; ++c) {
                    relres[c] = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
                    const bool need = relres[c] > opts->tol && iters[c] < opts->maxit;
                    cap[c] = need ? std::min(opts->maxit - iters[c], opts->restart) : 0;
                    // the correction needs to reduce this residual only by tol / relres
                    // (with a margin of 1/2), and never by more than inner_tol
                    itol[c] = relres[c] > 0 ? std::max(opts->inner_tol, 0.5 * opts->tol / relres[c]) : opts->inner_tol;
                    itol[c] = std::min(itol[c], 0.5);
                    any = any || need;
                }
                if (!any) break;
                if (solve_log()) {
                    double worst = 0.0;
                    int itmax = 0;
                    for (int c = 0; c < r; ++c) {
                        worst = std::max(worst, relres[c]);
                        itmax = std::max(itmax, iters[c]);
                    }
                    std::fprintf(stderr, "[igaefie] refinement step: FP64 max relres %.3e, iterations %d, inner "
                                         "precision %d\n", worst, itmax, cur);
                    std::fflush(stderr);
                }
                IGE_HIP(hipMemsetAsync(op->d_D.p, 0, sizeof(double2) * r * N, s));
                // columns already converged get an inner budget of 0 and a zero correction
                gmres_batched(op, r, op->d_r.p, op->d_D.p, itol, opts->restart, cap, cur, go, inner_b32, &ag_inner);
                ige::launch_axpby(op, (int64_t)r * N, make_double2(1, 0), op->d_D.p, make_double2(1, 0), X);
                for (int c = 0; c < r; ++c) {
                    iters[c] += go.iters[c];
                    if (cap[c] > 0) outer[c]++;
                    prev[c] = relres[c];
                    est[c] = go.relres_est[c];
                    lastcap[c] = cap[c];
                }
            }
        }
        // true FP64 relative residual of every column
        if (op->d_r.n < (size_t)r * N) op->d_r.alloc((size_t)r * N);
        if (op->d_red.n < (size_t)2 * r) op->d_red.alloc(2 * r);
        apply_dev(op, r, X, op->d_r.p, IGE_F64);
        ige::launch_axpby(op, (int64_t)r * N, make_double2(1, 0), F, make_double2(-1, 0), op->d_r.p);
        std::vector<double> rn(r), fn(r);
        ige::launch_norm2_b(op, r, op->d_r.p, op->d_red.p);
        ige::launch_norm2_b(op, r, F, op->d_red.p + r);
        IGE_HIP(hipMemcpyAsync(rn.data(), op->d_red.p, sizeof(double) * r, hipMemcpyDeviceToHost, s));
        IGE_HIP(hipMemcpyAsync(fn.data(), op->d_red.p + r, sizeof(double) * r, hipMemcpyDeviceToHost, s));
        if (ptr_kind == IGE_HOST)
            IGE_HIP(hipMemcpyAsync(x, X, sizeof(double2) * r * N, hipMemcpyDeviceToHost, s));
        IGE_HIP(hipStreamSynchronize(s));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int c = 0; c < r; ++c) {
            relres[c] = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
            // a converged estimate within rounding of tol counts as converged
            if (relres[c] > opts->tol * 1.05) notconv = true;
            if (stats) {
                stats[c].iters = iters[c];
                stats[c].outer = outer[c];
                stats[c].relres = relres[c];
                stats[c].seconds = secs;
            }
        }
    });
    if (rc == IGE_OK && notconv) {
        g_err = "GMRES reached maxit before the tolerance";
        return IGE_ENOTCONV;
    }
    return rc;
}

int ige_potential(ige_op op, int r, const ige_c64 *w, int ptr_kind, int npts, const double *points, ige_c64 *E)
{
    return guard([&] {
        IGE_REQUIRE(op && w && r >= 1 && npts >= 0 && (npts == 0 || (points && E)), "bad potential arguments");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        IGE_REQUIRE(ptr_kind == IGE_HOST || ptr_kind == IGE_DEVICE, "bad ptr_kind");
        for (int64_t i = 0; i < 3 * (int64_t)npts; ++i) IGE_REQUIRE(std::isfinite(points[i]), "non-finite point");
        set_device(op->ctx);
        hipStream_t s = op->ctx->stream;
        const int64_t N = op->D.N;
        ige::DBuf<double2> dw, dout;
        ige::DBuf<double> dpts, dsrc;
        dsrc.alloc(ige::potential_source_doubles(op));
        dpts.alloc(std::max<size_t>(1, (size_t)3 * npts));
        dout.alloc(std::max<size_t>(1, (size_t)3 * npts));
        if (npts) IGE_HIP(hipMemcpyAsync(dpts.p, points, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, s));
        const double2 *W = reinterpret_cast<const double2 *>(w);
        if (ptr_kind == IGE_HOST) {
            dw.alloc((size_t)r * N);
            IGE_HIP(hipMemcpyAsync(dw.p, w, sizeof(double2) * r * N, hipMemcpyHostToDevice, s));
            W = dw.p;
        }
        for (int c = 0; c < r; ++c) {
            ige::launch_potential(op, W + (size_t)c * N, npts, dpts.p, dout.p, dsrc.p);
            if (npts)
                IGE_HIP(hipMemcpyAsync(E + (size_t)c * 3 * npts, dout.p, sizeof(double2) * 3 * npts,
                                       hipMemcpyDeviceToHost, s));
        }
        IGE_HIP(hipStreamSynchronize(s));
    });
}

int ige_potential_noalloc(ige_op op, int r, const ige_c64 *w, int npts, const double *points, ige_c64 *E)
{
    return guard([&] {
        IGE_REQUIRE(op && w && r >= 1 && npts >= 0 && (npts == 0 || (points && E)), "bad potential arguments");
        IGE_REQUIRE(op->assembled, "operator was planned, not assembled");
        const size_t need = ige::potential_source_doubles(op);
        const size_t cap = ige::potential_scratch_doubles();
        if (need > cap)
            throw ige::Status{IGE_EINVAL, "operator too large for the fixed potential scratch: " +
                                              std::to_string(need * 8) + " bytes of source data > " +
                                              std::to_string(cap * 8)};
        set_device(op->ctx);
        double *scr = ige::potential_scratch(op->ctx->device);
        IGE_REQUIRE(scr != nullptr, "potential scratch not set up on this device");
        const int64_t N = op->D.N;
        const double2 *W = reinterpret_cast<const double2 *>(w);
        double2 *out = reinterpret_cast<double2 *>(E);
        for (int c = 0; c < r; ++c)
            ige::launch_potential(op, W + (size_t)c * N, npts, points, out + (size_t)c * 3 * npts, scr);
    });
}

int ige_peak_probe(ige_ctx ctx, int kind, double *value)
{
    return guard([&] {
        IGE_REQUIRE(ctx && value, "null argument");
        IGE_REQUIRE(ctx->device >= 0, "the probe needs a device context");
        IGE_REQUIRE(kind >= IGE_PROBE_HBM && kind <= IGE_PROBE_MFMA_F64, "bad probe kind");
        set_device(ctx);
        *value = ige::peak_probe(ctx->stream, kind);
    });
}

int ige_helmholtz_eval(ige_ctx ctx, int64_t n, double kappa, const double *r2, ige_c64 *out, int prec)
{
    return guard([&] {
        IGE_REQUIRE(ctx && r2 && out && n >= 0, "bad arguments");
        IGE_REQUIRE(ctx->device >= 0, "needs a device context");
        IGE_REQUIRE(std::isfinite(kappa) && kappa > 0.0, "kappa must be positive");
        for (int64_t i = 0; i < n; ++i) IGE_REQUIRE(std::isfinite(r2[i]) && r2[i] > 0.0, "r2 must be positive");
        if (n == 0) return;
        set_device(ctx);
        DBuf<double> dr;
        DBuf<double2> dout, dtab;
        dr.alloc(n);
        dout.alloc(n);
        IGE_HIP(hipMemcpyAsync(dr.p, r2, sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
        dtab.upload(sincos_table(), ctx->stream);
        IGE_REQUIRE(prec == IGE_F64 || prec == IGE_F32, "bad precision");
        ige::launch_helmholtz_eval(ctx->stream, n, kappa, dr.p, dout.p, prec, dtab.p);
        IGE_HIP(hipMemcpyAsync(out, dout.p, sizeof(double2) * n, hipMemcpyDeviceToHost, ctx->stream));
        IGE_HIP(hipStreamSynchronize(ctx->stream));
    });
}

}  // extern "C"
