// HIP kernels of the igaefie library (gfx950, wave64), by step of the path:
//
//   geometry   element_data / node_geometry : geometry from the rational Bezier form at
//              the regular Gauss points of every element and at the Chebyshev nodes of
//              every cluster
//   near field near_regular / near_singular : element-pair Galerkin quadrature,
//              accumulated into dense blocks over leaf function slots (regular pairs on
//              the FP64 matrix cores)
//   P2M        leaf moments, fused with the gather x_super = T x (1-D factors of T)
//   M2M        upward transfer of the moments (nested cluster bases)
//   M2L        coupling of admissible cluster pairs with the interpolated kernel
//   L2L        downward transfer
//   L2P        test-side moments, fused with the scatter T^T
//   near product near_blk + near_gather: product with the stored blocks and their
//              transposes, then a fixed-order sum per unknown
//   rhs        plane-wave right-hand side
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "device_math.hpp"
#include "op.hpp"

namespace ige {

namespace {

constexpr int kWave = 64;
typedef double dx4 __attribute__((ext_vector_type(4)));   // FP64 matrix-core accumulator
__device__ __constant__ double kInv4Pi = 0.07957747154594767;   // 1/(4 pi)

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
using dm::surf_elem;

// Helmholtz kernel e^{i k r} / (4 pi r) (library sincos, correctly rounded sqrt):
// used by the assembly kernels
__device__ inline double2 helmholtz(double kappa, double r)
{
    double sn, cs;
    sincos(kappa * r, &sn, &cs);
    const double f = kInv4Pi / r;
    return make_double2(cs * f, sn * f);
}

// Bernstein values and derivatives of degree deg <= kMaxP at x
__device__ inline void bernstein(int deg, double x, double *B, double *D)
{
    double T[kMaxP + 1];
    T[0] = 1.0;
    for (int k = 1; k < deg; ++k) {
        T[k] = x * T[k - 1];
        for (int i = k - 1; i >= 1; --i) T[i] = (1.0 - x) * T[i] + x * T[i - 1];
        T[0] = (1.0 - x) * T[0];
    }
    if (deg == 0) {
        B[0] = 1.0;
        D[0] = 0.0;
        return;
    }
    for (int i = 0; i <= deg; ++i) {
        const double lo = (i >= 1) ? T[i - 1] : 0.0;
        const double hi = (i <= deg - 1) ? T[i] : 0.0;
        D[i] = deg * (lo - hi);
        B[i] = (1.0 - x) * hi + x * lo;
    }
}

// 1-D spline pieces on element e at element-local x: degree p values/derivatives
// (derivatives w.r.t. the patch parameter) and degree p-1 values
__device__ inline void spline_pieces(const DevOp &o, int e, double x, double *Pv, double *Pd, double *Qv)
{
    const int p = o.p;
    double B[kMaxP + 1], D[kMaxP + 1];
    bernstein(p, x, B, D);
    for (int t = 0; t <= p; ++t) {
        double v = 0.0, d = 0.0;
        const double *c = o.ext_p + ((size_t)e * (p + 1) + t) * (p + 1);
        for (int a = 0; a <= p; ++a) {
            v += c[a] * B[a];
            d += c[a] * D[a];
        }
        Pv[t] = v;
        Pd[t] = d / o.h;
    }
    double Bq[kMaxP + 1], Dq[kMaxP + 1];
    bernstein(p - 1, x, Bq, Dq);
    for (int t = 0; t < p; ++t) {
        double v = 0.0;
        const double *c = o.ext_q + ((size_t)e * p + t) * p;
        for (int a = 0; a < p; ++a) v += c[a] * Bq[a];
        Qv[t] = v;
    }
}

// Fixed-degree variants (fully unrolled, no scratch): Bernstein values and
// derivatives, spline pieces and rational Bezier patch evaluation.
template <int DEG>
__device__ inline void bernstein_t(double x, double *B, double *D)
{
    if constexpr (DEG == 0) {
        B[0] = 1.0;
        D[0] = 0.0;
    } else {
        double T[DEG];
        T[0] = 1.0;
#pragma unroll
        for (int k = 1; k < DEG; ++k) {
            T[k] = x * T[k - 1];
#pragma unroll
            for (int i = k - 1; i >= 1; --i) T[i] = (1.0 - x) * T[i] + x * T[i - 1];
            T[0] = (1.0 - x) * T[0];
        }
#pragma unroll
        for (int i = 0; i <= DEG; ++i) {
            const double lo = (i >= 1) ? T[i >= 1 ? i - 1 : 0] : 0.0;
            const double hi = (i <= DEG - 1) ? T[i <= DEG - 1 ? i : 0] : 0.0;
            D[i] = DEG * (lo - hi);
            B[i] = (1.0 - x) * hi + x * lo;
        }
    }
}

template <int P>
__device__ inline void spline_pieces_t(const DevOp &o, int e, double x, double *Pv, double *Pd, double *Qv)
{
    double B[P + 1], D[P + 1];
    bernstein_t<P>(x, B, D);
#pragma unroll
    for (int t = 0; t <= P; ++t) {
        double v = 0.0, d = 0.0;
        const double *c = o.ext_p + ((size_t)e * (P + 1) + t) * (P + 1);
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            v += c[a] * B[a];
            d += c[a] * D[a];
        }
        Pv[t] = v;
        Pd[t] = d / o.h;
    }
    double Bq[P], Dq[P];
    bernstein_t<P - 1>(x, Bq, Dq);
#pragma unroll
    for (int t = 0; t < P; ++t) {
        double v = 0.0;
        const double *c = o.ext_q + ((size_t)e * P + t) * P;
#pragma unroll
        for (int a = 0; a < P; ++a) v += c[a] * Bq[a];
        Qv[t] = v;
    }
}

template <int PU, int PV>
__device__ inline void bezier_eval_t(const GeomView &g, const PatchHdr &h, double u, double v, double X[3],
                                     double Xu[3], double Xv[3])
{
    int su = 0, sv = 0;
    while (su < h.su - 1 && u >= g.brk[h.brk_u + su + 1]) ++su;
    while (sv < h.sv - 1 && v >= g.brk[h.brk_v + sv + 1]) ++sv;
    const double ua = g.brk[h.brk_u + su], ub = g.brk[h.brk_u + su + 1];
    const double va = g.brk[h.brk_v + sv], vb = g.brk[h.brk_v + sv + 1];
    const double t = (u - ua) / (ub - ua), s = (v - va) / (vb - va);
    double Bu[PU + 1], Du[PU + 1], Bv[PV + 1], Dv[PV + 1];
    bernstein_t<PU>(t, Bu, Du);
    bernstein_t<PV>(s, Bv, Dv);
    const double *c = g.cp + h.cp + (size_t)(sv * h.su + su) * (PV + 1) * (PU + 1) * 4;
    double A[4] = {0, 0, 0, 0}, Au[4] = {0, 0, 0, 0}, Av[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j2 = 0; j2 <= PV; ++j2)
#pragma unroll
        for (int j1 = 0; j1 <= PU; ++j1) {
            const double *Pc = c + (j2 * (PU + 1) + j1) * 4;
            const double b = Bu[j1] * Bv[j2], bu = Du[j1] * Bv[j2], bv = Bu[j1] * Dv[j2];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                A[k] += b * Pc[k];
                Au[k] += bu * Pc[k];
                Av[k] += bv * Pc[k];
            }
        }
    const double iw = 1.0 / A[3], du = 1.0 / (ub - ua), dv = 1.0 / (vb - va);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        X[k] = A[k] * iw;
        Xu[k] = (Au[k] - X[k] * Au[3]) * iw * du;
        Xv[k] = (Av[k] - X[k] * Av[3]) * iw * dv;
    }
}

// other degrees: out of line, so that its stack arrays do not enlarge the callers
__device__ __noinline__ void geom_eval_generic(const GeomView &g, int j, double u, double v, double X[3], double Xu[3],
                                               double Xv[3])
{
    bezier_eval(g, j, u, v, X, Xu, Xv);
}

// patch evaluation with unrolled paths for bilinear and biquadratic patches
__device__ inline void geom_eval(const GeomView &g, int j, double u, double v, double X[3], double Xu[3], double Xv[3])
{
    const PatchHdr h = g.hdr[j];
    if (h.pu == 2 && h.pv == 2) bezier_eval_t<2, 2>(g, h, u, v, X, Xu, Xv);
    else if (h.pu == 1 && h.pv == 1) bezier_eval_t<1, 1>(g, h, u, v, X, Xu, Xv);
    else geom_eval_generic(g, j, u, v, X, Xu, Xv);
}

// local function l of an element: (component, t1, t2); the scalar operator has the
// (p+1)^2 tensor B-splines, t2 major, in component 0
__device__ inline void local_index(const DevOp &o, int l, int &a, int &t1, int &t2)
{
    const int p = o.p;
    if (o.scalar) {
        a = 0;
        t2 = l / (p + 1);
        t1 = l % (p + 1);
        return;
    }
    const int n0 = p * (p + 1);
    if (l < n0) {
        a = 0;
        t2 = l / (p + 1);
        t1 = l % (p + 1);
    } else {
        a = 1;
        const int r = l - n0;
        t2 = r / p;
        t1 = r % p;
    }
}

// values of the local functions at element-local (x, y): Phi (3) and div, unsigned
// (scalar operator: Phi = 0 and the value times the surface element in place of div)
template <int NL>
__device__ inline void local_values(const DevOp &o, int e1, int e2, double x, double y, const double Fu[3],
                                    const double Fv[3], double Phi[NL][3], double Dv[NL])
{
    double Pu[kMaxP + 1], dPu[kMaxP + 1], Qu[kMaxP + 1], Pv[kMaxP + 1], dPv[kMaxP + 1], Qv[kMaxP + 1];
    spline_pieces(o, e1, x, Pu, dPu, Qu);
    spline_pieces(o, e2, y, Pv, dPv, Qv);
    if (o.scalar) {   // value times the surface element, no field part
        const double J = surf_elem(Fu, Fv);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            int a, t1, t2;
            local_index(o, l, a, t1, t2);
            Phi[l][0] = Phi[l][1] = Phi[l][2] = 0.0;
            Dv[l] = Pu[t1] * Pv[t2] * J;
        }
        return;
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        int a, t1, t2;
        local_index(o, l, a, t1, t2);
        double val, div;
        if (a == 0) {
            val = Pu[t1] * Qv[t2];
            div = dPu[t1] * Qv[t2];
        } else {
            val = Qu[t1] * Pv[t2];
            div = Qu[t1] * dPv[t2];
        }
        const double *F = (a == 0) ? Fu : Fv;
        Phi[l][0] = val * F[0];
        Phi[l][1] = val * F[1];
        Phi[l][2] = val * F[2];
        Dv[l] = div;
    }
}

// The same values written straight to a row of shared memory: (Phi_l, cdiv * div_l).
template <int NL>
__device__ inline void local_values_lds(const DevOp &o, int e1, int e2, double x, double y, const double Fu[3],
                                        const double Fv[3], double cdiv, double (*dst)[4])
{
    double Pu[kMaxP + 1], dPu[kMaxP + 1], Qu[kMaxP + 1], Pv[kMaxP + 1], dPv[kMaxP + 1], Qv[kMaxP + 1];
    spline_pieces(o, e1, x, Pu, dPu, Qu);
    spline_pieces(o, e2, y, Pv, dPv, Qv);
    if (o.scalar) {
        const double J = surf_elem(Fu, Fv);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            int a, t1, t2;
            local_index(o, l, a, t1, t2);
            dst[l][0] = dst[l][1] = dst[l][2] = 0.0;
            dst[l][3] = cdiv * Pu[t1] * Pv[t2] * J;
        }
        return;
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        int a, t1, t2;
        local_index(o, l, a, t1, t2);
        double val, div;
        if (a == 0) {
            val = Pu[t1] * Qv[t2];
            div = dPu[t1] * Qv[t2];
        } else {
            val = Qu[t1] * Pv[t2];
            div = Qu[t1] * dPv[t2];
        }
        const double *F = (a == 0) ? Fu : Fv;
        dst[l][0] = val * F[0];
        dst[l][1] = val * F[1];
        dst[l][2] = val * F[2];
        dst[l][3] = cdiv * div;
    }
}

// (Phi_l, cdiv * div_l) for the NL = 2P(P+1) local functions, into rows of shared memory
template <int P, bool SC = false>
__device__ inline void local_values_lds_t(const DevOp &o, int e1, int e2, double x, double y, const double Fu[3],
                                          const double Fv[3], double cdiv, double (*dst)[4])
{
    constexpr int NL = 2 * P * (P + 1);
    double Pu[P + 1], dPu[P + 1], Qu[P], Pv[P + 1], dPv[P + 1], Qv[P];
    spline_pieces_t<P>(o, e1, x, Pu, dPu, Qu);
    spline_pieces_t<P>(o, e2, y, Pv, dPv, Qv);
    if constexpr (SC) {   // scalar: (p+1)^2 tensor B-splines, value times |J| in slot 3
        const double J = surf_elem(Fu, Fv);
#pragma unroll
        for (int l = 0; l < (P + 1) * (P + 1); ++l) {
            dst[l][0] = dst[l][1] = dst[l][2] = 0.0;
            dst[l][3] = cdiv * Pu[l % (P + 1)] * Pv[l / (P + 1)] * J;
        }
        return;
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const bool a0 = l < P * (P + 1);
        const int r = a0 ? l : l - P * (P + 1);
        const int t2 = a0 ? r / (P + 1) : r / P, t1 = a0 ? r % (P + 1) : r % P;
        const double val = a0 ? Pu[t1] * Qv[t2] : Qu[t1] * Pv[t2];
        const double div = a0 ? dPu[t1] * Qv[t2] : Qu[t1] * dPv[t2];
        const double *F = a0 ? Fu : Fv;
        dst[l][0] = val * F[0];
        dst[l][1] = val * F[1];
        dst[l][2] = val * F[2];
        dst[l][3] = cdiv * div;
    }
}

__device__ inline void elem_of(const DevOp &o, int64_t e, int &j, int &e1, int &e2)
{
    const int nn = o.n * o.n;
    j = (int)(e / nn);
    const int r = (int)(e % nn);
    e2 = r / o.n;
    e1 = r % o.n;
}

__device__ inline void local_dof(const DevOp &o, int j, int e1, int e2, int l, int &idx, double &sg)
{
    int a, t1, t2;
    local_index(o, l, a, t1, t2);
    const size_t off = (((size_t)j * 2 + a) * o.nb + (e2 + t2)) * o.nb + (e1 + t1);
    idx = o.dof[off];
    sg = (double)o.sgn[off];
}

// FP64 matrix-core instruction 16x16x4: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register j of lane l holds D[l / 16 + 4 j][l % 16].
// Operand order: for step t a lane supplies the entry with quadrature index
// q = frag_q(t, lane) in reduction slot lane / 16, so that accumulator register j of
// a first product over tile qt is the operand of step t = 4 qt + j of a second.
__device__ inline int frag_q(int t, int lane) { return 16 * (t >> 2) + 4 * (t & 3) + (lane >> 4); }

// ---------------------------------------------------------------------------
// a0: element data at the regular Gauss points
// ---------------------------------------------------------------------------
// ePsiF[e][c][lt][t][lane] = ePsi[e][c][16 lt + lane % 16][frag_q(t, lane)] (zero padded
// to 16-row tiles in l and to 4*QT steps in q, QT = ceil(G2 / 16))
template <int NL>
__global__ void k_element_data(DevOp o, double *eX, double *ePsi, double *ePsiF, double *eC)
{
    const int64_t e = blockIdx.x;
    int j, e1, e2;
    elem_of(o, e, j, e1, e2);
    const int G2 = o.G2;
    for (int q = threadIdx.x; q < G2; q += blockDim.x) {
        const int a = q % o.g, b = q / o.g;
        const double x = o.gx[a], y = o.gx[b];
        const double u = (e1 + x) * o.h, v = (e2 + y) * o.h;
        double X[3], Fu[3], Fv[3];
        bezier_eval(o.geo, j, u, v, X, Fu, Fv);
        const double w = o.gw[a] * o.gw[b] * o.h * o.h;
        double Phi[NL][3], Dv[NL];
        local_values<NL>(o, e1, e2, x, y, Fu, Fv, Phi, Dv);
        for (int d = 0; d < 3; ++d) eX[((size_t)e * 3 + d) * G2 + q] = X[d];
        constexpr int LT = (NL + 15) / 16;
        const int T = 4 * ((G2 + 15) / 16);
        const int t = 4 * (q / 16) + (q % 16) / 4, lq = 16 * (q % 4);
        double *F = ePsiF + (size_t)e * 4 * LT * T * 64;
        for (int l = 0; l < NL; ++l) {
            for (int d = 0; d < 3; ++d) ePsi[(((size_t)e * 4 + d) * NL + l) * G2 + q] = w * Phi[l][d];
            ePsi[(((size_t)e * 4 + 3) * NL + l) * G2 + q] = w * Dv[l];
            const int lt = l / 16, lane = l % 16 + lq;
            for (int d = 0; d < 3; ++d) F[((d * LT + lt) * T + t) * 64 + lane] = w * Phi[l][d];
            F[((3 * LT + lt) * T + t) * 64 + lane] = w * Dv[l];
        }
    }
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        const int cu = (k == 1 || k == 2) ? 1 : 0, cv = (k >= 2) ? 1 : 0;
        double X[3], Fu[3], Fv[3];
        bezier_eval(o.geo, j, (e1 + cu) * o.h, (e2 + cv) * o.h, X, Fu, Fv);
        for (int d = 0; d < 3; ++d) eC[(size_t)e * 12 + k * 3 + d] = X[d];
    }
}

// a0: geometry at the Chebyshev nodes of every cluster
__global__ void k_node_geometry(DevOp o, int NC, double *nodeX, double *nodeT)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NC * o.Q) return;
    const int gc = (int)(t / o.Q), mm = (int)(t % o.Q);
    int lvl = 0;
    while (lvl < o.L && gc >= o.lvl_off[lvl + 1]) ++lvl;
    const int id = gc - (int)o.lvl_off[lvl];
    const int S = 1 << lvl;
    const int j = id / (S * S), r = id % (S * S), k2 = r / S, k1 = r % S;
    // the nodes of the level's degree (stored with the stride of the largest degree)
    const int Q1l = o.ql[lvl] + 1;
    if (mm >= Q1l * Q1l) return;
    const int m1 = mm % Q1l, m2 = mm / Q1l;
    const double *xn = o.xnl + (size_t)lvl * kMaxQ1;
    const double H = 1.0 / S;
    double X[3], Fu[3], Fv[3];
    bezier_eval(o.geo, j, (k1 + xn[m1]) * H, (k2 + xn[m2]) * H, X, Fu, Fv);
    for (int d = 0; d < 3; ++d) {
        nodeX[((size_t)gc * 3 + d) * o.Q + mm] = X[d];
        nodeT[((size_t)gc * 6 + d) * o.Q + mm] = Fu[d];
        nodeT[((size_t)gc * 6 + 3 + d) * o.Q + mm] = Fv[d];
    }
}

__device__ inline bool share_corner(const DevOp &o, int64_t e, int64_t f)
{
    const double *A = o.eC + e * 12, *B = o.eC + f * 12;
    for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) {
            const double d0 = A[3 * x] - B[3 * y], d1 = A[3 * x + 1] - B[3 * y + 1], d2 = A[3 * x + 2] - B[3 * y + 2];
            if (sqrt(d0 * d0 + d1 * d1 + d2 * d2) <= o.scale_tol) return true;
        }
    return false;
}

// row tiles of test functions per workgroup of k_near_regular: all up to 24 local
// functions, one 16-row tile for more (p = 4: 40 functions, three workgroups)
constexpr int near_regular_lr(int nl) { return nl <= 24 ? (nl + 15) / 16 : 1; }

// ---------------------------------------------------------------------------
// a1: regular element pairs (no shared corner).  With S = (1, 1, 1, -kappa^-2) and
// the weights folded into Psi,
//   B[l][l'] = sum_c S_c sum_q Psi_e^c[l][q] sum_q' K(q, q') Psi_f^c[l'][q'],
// computed as two products on the FP64 matrix cores per trial element f:
//   Y_c(q', l) = sum_q K(q, q') Psi_e^c[l][q]      (K as operand A, Psi_e as B)
//   B(l, l') += sum_q' Y_c(q', l) Psi_f^c[l'][q']  (Y from the accumulators as A)
// The accumulator layout of the first product (row lane/16 + 4 j) is the operand
// layout of the second when its reduction slots are ordered by frag_q.
// A workgroup takes one block, one test element e of the target leaf and a square
// of sb x sb trial elements of the source leaf.  The four waves take the trial
// elements four at a time; their element-pair blocks are added to the block rows of
// e in shared memory one wave after the other (trial elements in ascending order),
// then the element pairs of e that share a corner with a trial element of the square
// (computed before by k_near_singular) in list order.  Every sum therefore has a
// fixed order.
// Launched once per colour: the test elements of a launch are p + 1 apart in both
// directions (no glued function in common, so no block row in common), and with
// several trial squares per leaf the squares of a launch are two apart (sb >= p: no
// column in common).  Each block entry thus has at most one writer per launch, and
// the launches run in a fixed order on one stream: the assembled blocks are the same
// bits on every run.
// ---------------------------------------------------------------------------
template <int NL, int QT, int LR>
__device__ __forceinline__ void near_regular_body(const DevOp &o, int sb, int ce1, int ce2, int cs1, int cs2, int sstep)
{
    // LR of the LT 16-row tiles of test functions per workgroup (LR = LT: all rows;
    // otherwise the rows are split over LT / LR workgroups, for the larger degrees)
    constexpr int LT = (NL + 15) / 16, T = 4 * QT, NRT = LT / LR;
    constexpr int NR = LR == LT ? NL : 16 * LR;       // test-function rows of this workgroup
    extern __shared__ double2 sacc[];                 // [NR][2 Wsb^2], then [4][NR][NL] staging
    __shared__ double sXe[3][16 * QT];                // test element points (zero padded)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int s = o.s, nsb = s / sb, Wsb = sb + o.p, nslot = 2 * Wsb * Wsb, P1 = o.p + 1;
    double2 *sstage = sacc + NR * nslot;
    // test elements and trial squares of this colour
    const int n1 = (s - ce1 + P1 - 1) / P1, n2 = (s - ce2 + P1 - 1) / P1;
    const int m1 = (nsb - cs1 + sstep - 1) / sstep, m2 = (nsb - cs2 + sstep - 1) / sstep;
    int64_t blk = blockIdx.x;
    const int u0 = LR * (int)(blk % NRT);             // first row tile
    blk /= NRT;
    const int l0 = 16 * u0;                           // first test function
    const int sub = (int)(blk % (m1 * m2));
    blk /= m1 * m2;
    const int tc = (int)(blk % (n1 * n2));
    const int64_t b = blk / (n1 * n2);
    const int lt = o.bpair[2 * b], ls = o.bpair[2 * b + 1];
    const int SL = o.SL;
    const int jt = lt / (SL * SL), jr = lt % (SL * SL), js = ls / (SL * SL), jsr = ls % (SL * SL);
    const int tl1 = ce1 + P1 * (tc % n1), tl2 = ce2 + P1 * (tc / n1);   // e inside its leaf
    const int ti = tl2 * s + tl1;
    const int te1 = (jr % SL) * s + tl1, te2 = (jr / SL) * s + tl2;
    const int sl1 = (cs1 + sstep * (sub % m1)) * sb, sl2 = (cs2 + sstep * (sub / m1)) * sb;   // trial square
    const int fx0 = (jsr % SL) * s + sl1, fy0 = (jsr / SL) * s + sl2;
    const int64_t e = ((int64_t)jt * o.n + te2) * o.n + te1;
    const int G2 = o.G2;
    for (int i = threadIdx.x; i < NR * nslot; i += blockDim.x) sacc[i] = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < 3 * 16 * QT; i += blockDim.x) {
        const int d = i / (16 * QT), q = i % (16 * QT);
        sXe[d][q] = q < G2 ? o.eX[(e * 3 + d) * G2 + q] : 0.0;
    }
    constexpr size_t FE = (size_t)4 * LT * T * 64;
    double pa[4][LR][T];
    {
        const double *Fe = o.ePsiF + (size_t)e * FE;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int u = 0; u < LR; ++u)
#pragma unroll
                for (int t = 0; t < T; ++t)
                    pa[c][u][t] = Fe[((c * LT + u0 + u) * T + t) * 64 + lane] * (c == 3 ? o.cdiv : 1.0);
    }
    __syncthreads();
    const int nfe = sb * sb, nround = (nfe + 3) / 4;
    for (int rd = 0; rd < nround; ++rd) {
        const int fi = 4 * rd + wv;
        const int fe1 = fx0 + fi % sb, fe2 = fy0 + fi / sb;
        const int64_t f = ((int64_t)js * o.n + fe2) * o.n + fe1;
        // wave-uniform: trial element exists and shares no corner with e (those pairs
        // come from the singular kernel)
        const bool act = fi < nfe && !share_corner(o, e, f);
        dx4 br[LR][LT], bi[LR][LT];
        if (act) {
#pragma unroll
            for (int u = 0; u < LR; ++u)
#pragma unroll
                for (int v = 0; v < LT; ++v) {
                    br[u][v] = dx4{0.0, 0.0, 0.0, 0.0};
                    bi[u][v] = dx4{0.0, 0.0, 0.0, 0.0};
                }
            // kernel values as operand A: row q' = 16 qt + lane % 16, slot q = frag_q(t, lane)
            double kre[QT][T], kim[QT][T];
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
                const int qb = 16 * qt + (lane & 15);
                const bool okb = qb < G2;
                double xb0 = 0.0, xb1 = 0.0, xb2 = 0.0;
                if (okb) {
                    xb0 = o.eX[(f * 3 + 0) * G2 + qb];
                    xb1 = o.eX[(f * 3 + 1) * G2 + qb];
                    xb2 = o.eX[(f * 3 + 2) * G2 + qb];
                }
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const int qa = frag_q(t, lane);
                    double2 K = make_double2(0.0, 0.0);
                    if (okb && qa < G2) {
                        const double d0 = sXe[0][qa] - xb0, d1 = sXe[1][qa] - xb1, d2 = sXe[2][qa] - xb2;
                        K = dm::helmholtz_r2(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2)));
                    }
                    kre[qt][t] = K.x;
                    kim[qt][t] = K.y;
                }
            }
            const double *Ff = o.ePsiF + (size_t)f * FE;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                dx4 yr[QT][LR], yi[QT][LR];
#pragma unroll
                for (int qt = 0; qt < QT; ++qt)
#pragma unroll
                    for (int u = 0; u < LR; ++u) {
                        yr[qt][u] = dx4{0.0, 0.0, 0.0, 0.0};
                        yi[qt][u] = dx4{0.0, 0.0, 0.0, 0.0};
                    }
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int qt = 0; qt < QT; ++qt)
#pragma unroll
                        for (int u = 0; u < LR; ++u) {
                            yr[qt][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(kre[qt][t], pa[c][u][t], yr[qt][u], 0, 0, 0);
                            yi[qt][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(kim[qt][t], pa[c][u][t], yi[qt][u], 0, 0, 0);
                        }
#pragma unroll
                for (int v = 0; v < LT; ++v)
#pragma unroll
                    for (int qt = 0; qt < QT; ++qt)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const double pb = Ff[((c * LT + v) * T + 4 * qt + j) * 64 + lane];
#pragma unroll
                            for (int u = 0; u < LR; ++u) {
                                br[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(yr[qt][u][j], pb, br[u][v], 0, 0, 0);
                                bi[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(yi[qt][u][j], pb, bi[u][v], 0, 0, 0);
                            }
                        }
            }
        }
        // rows l = 16 u + lane / 16 + 4 j, columns l' = 16 v + lane % 16 into this wave's
        // staging block, then the four staged blocks are added in wave order
        double2 *stg = sstage + (size_t)wv * NR * NL;
        if (act) {
#pragma unroll
            for (int v = 0; v < LT; ++v) {
                const int lb = 16 * v + (lane & 15);
#pragma unroll
                for (int u = 0; u < LR; ++u)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int lr = 16 * u + (lane >> 4) + 4 * j;   // row of this workgroup
                        if (l0 + lr < NL && lb < NL) stg[lr * NL + lb] = make_double2(br[u][v][j], bi[u][v][j]);
                    }
            }
        }
        __syncthreads();
        for (int w = 0; w < 4; ++w) {
            const int fw = 4 * rd + w;
            // uniform over the workgroup: whether wave w computed a pair this round
            const bool aw = fw < nfe && !share_corner(o, e, ((int64_t)js * o.n + fy0 + fw / sb) * o.n + fx0 + fw % sb);
            if (aw) {
                const int q1 = fw % sb, q2 = fw / sb;
                const double2 *sw = sstage + (size_t)w * NR * NL;
                for (int i = threadIdx.x; i < NR * NL; i += blockDim.x) {
                    const int l = i / NL, lb = i % NL;
                    if (l0 + l >= NL) continue;
                    int a, t1, t2;
                    local_index(o, lb, a, t1, t2);
                    const int slot = a * Wsb * Wsb + (q2 + t2) * Wsb + (q1 + t1);
                    const double2 v = sw[i];
                    double2 &acc = sacc[l * nslot + slot];
                    acc.x += v.x;
                    acc.y += v.y;
                }
            }
            __syncthreads();
        }
    }
    // element pairs of e with a shared corner whose trial element lies in the square
    const int kb = o.sing_ptr[b * (int64_t)(s * s) + ti], ke = o.sing_ptr[b * (int64_t)(s * s) + ti + 1];
    for (int k = kb; k < ke; ++k) {
        const int64_t f = o.sing[k].f;
        int jf, f1, f2;
        elem_of(o, f, jf, f1, f2);
        const int q1 = f1 - fx0, q2 = f2 - fy0;
        if (q1 < 0 || q1 >= sb || q2 < 0 || q2 >= sb) continue;   // uniform over the workgroup
        const double2 *P = o.sblk + (size_t)k * NL * NL + (size_t)l0 * NL;
        for (int i = threadIdx.x; i < NR * NL; i += blockDim.x) {
            const int l = i / NL, lb = i % NL;
            if (l0 + l >= NL) continue;
            int a, t1, t2;
            local_index(o, lb, a, t1, t2);
            const int slot = a * Wsb * Wsb + (q2 + t2) * Wsb + (q1 + t1);
            const double2 v = P[i];
            double2 &acc = sacc[l * nslot + slot];
            acc.x += v.x;
            acc.y += v.y;
        }
        __syncthreads();
    }
    const int W = o.W, nF = o.nF;
    for (int i = threadIdx.x; i < NR * nslot; i += blockDim.x) {
        const double2 v = sacc[i];
        if (v.x == 0.0 && v.y == 0.0) continue;
        const int l = l0 + i / nslot, sl = i % nslot;
        if (l >= NL) continue;
        const int a = sl / (Wsb * Wsb), r = sl % (Wsb * Wsb);
        const int i1 = sl1 + r % Wsb, i2 = sl2 + r / Wsb;
        if (i1 >= (a == 0 ? W : W - 1) || i2 >= ((a == 0 && !o.scalar) ? W - 1 : W)) {
            atomicAdd(o.err, 1);
            continue;
        }
        const int kc = leaf_slot(W, a, i1, i2);
        int ar, t1, t2;
        local_index(o, l, ar, t1, t2);
        const int kr = leaf_slot(W, ar, tl1 + t1, tl2 + t2);
        // signs of the glued unknowns folded in; slots without an unknown are skipped
        const double sg = (double)o.leafsgn[(size_t)lt * nF + kr] * (double)o.leafsgn[(size_t)ls * nF + kc];
        if (sg == 0.0) continue;
        double2 *dst = o.bval + ((size_t)b * nF + kr) * nF + kc;   // the only writer in this launch
        double2 cur = *dst;
        cur.x += sg * v.x;
        cur.y += sg * v.y;
        *dst = cur;
    }
}

// the small rules (one or two 16-point tiles, up to 12 local functions) fit two
// workgroups per CU without spilling; the others take all registers of one
template <int NL, int QT>
__global__ __launch_bounds__(256) void k_near_regular(DevOp o, int sb, int ce1, int ce2, int cs1, int cs2, int sstep)
{
    near_regular_body<NL, QT, near_regular_lr(NL)>(o, sb, ce1, ce2, cs1, cs2, sstep);
}
template <int NL, int QT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_near_regular_o2(DevOp o, int sb, int ce1,
                                                                                                   int ce2, int cs1, int cs2,
                                                                                                   int sstep)
{
    near_regular_body<NL, QT, near_regular_lr(NL)>(o, sb, ce1, ce2, cs1, cs2, sstep);
}

// ---------------------------------------------------------------------------
// a1: element pairs sharing a corner (relative-coordinate / Duffy sub-rules),
// one wavefront per pair; each pair's NL x NL block is written to its own slot of a
// scratch array (no accumulation here).
// ---------------------------------------------------------------------------
__device__ inline void frame_map(int code, double c1, double c2, double &x, double &y)
{
    const int o1 = code & 1, o2 = (code >> 1) & 1, sw = (code >> 2) & 1;
    const double du = o1 ? -1.0 : 1.0, dv = o2 ? -1.0 : 1.0;
    if (!sw) {
        x = o1 + du * c1;
        y = o2 + dv * c2;
    } else {
        x = o1 + du * c2;
        y = o2 + dv * c1;
    }
}

// canonical point (s1, s2) on the test element, (t1, t2) on the trial element and
// weight of sub-rule point idx
__device__ inline void singular_point(const DevOp &o, int kind, int idx, double &s1, double &s2, double &t1,
                                      double &t2, double &wt)
{
    const int gs = o.gs, g4 = gs * gs * gs * gs;
    const int sub = idx / g4;
    int r = idx % g4;
    const int id = r % gs; r /= gs;
    const int ic = r % gs; r /= gs;
    const int ib = r % gs; r /= gs;
    const int ia = r;
    const double xi = o.sx[ia], y1 = o.sx[ib], y2 = o.sx[ic], y3 = o.sx[id];
    const double w4 = o.sw[ia] * o.sw[ib] * o.sw[ic] * o.sw[id];
    if (kind == 1) {
        // identical: per direction |x_k - y_k| = w_k with both orders; (w1, w2) triangle split
        const int tri = sub >> 2, sg1 = (sub >> 1) & 1, sg2 = sub & 1;
        const double w1 = tri == 0 ? xi : xi * y1;
        const double w2 = tri == 0 ? xi * y1 : xi;
        if (!sg1) { s1 = (1.0 - w1) * y2; t1 = s1 + w1; } else { t1 = (1.0 - w1) * y2; s1 = t1 + w1; }
        if (!sg2) { s2 = (1.0 - w2) * y3; t2 = s2 + w2; } else { t2 = (1.0 - w2) * y3; s2 = t2 + w2; }
        wt = w4 * xi * (1.0 - w1) * (1.0 - w2);
    } else if (kind == 2) {
        // common edge at s1 = t1 = 0: distances A, B to the edge and W = |s2 - t2|
        const int pyr = sub >> 1, sg = sub & 1;
        double A, B, W;
        if (pyr == 0) { A = xi; B = xi * y1; W = xi * y2; }
        else if (pyr == 1) { B = xi; A = xi * y1; W = xi * y2; }
        else { W = xi; A = xi * y1; B = xi * y2; }
        double a2, b2;
        if (!sg) { a2 = (1.0 - W) * y3; b2 = a2 + W; } else { b2 = (1.0 - W) * y3; a2 = b2 + W; }
        s1 = A; s2 = a2; t1 = B; t2 = b2;
        wt = w4 * xi * xi * (1.0 - W);
    } else {
        // common vertex at the origin of both: the largest of the four coordinates is xi
        double z[4];
        const double rest[3] = {xi * y1, xi * y2, xi * y3};
        int k = 0;
        for (int i = 0; i < 4; ++i) z[i] = (i == sub) ? xi : rest[k++];
        s1 = z[0]; s2 = z[1]; t1 = z[2]; t2 = z[3];
        wt = w4 * xi * xi * xi;
    }
}

// Singular pairs: one wave per pair.  The points of the sub-rules are processed in
// batches of 32: the lower half-wave evaluates geometry and local values on the
// test element, the upper half on the trial element, into shared memory; then
//   B[l][l'] += sum_q K_q sum_c Psi_a[q][l][c] Psi_b[q][l'][c]
// runs on the FP64 matrix cores with the four components c as the reduction slots
// of one instruction per point (K_q = weight * kernel folded into the test side).
template <int P, bool SC = false>
__global__ __launch_bounds__(64) void k_near_singular(DevOp o, const SingularPair *list)
{
    // points per batch: 32 (16 for p = 4, whose 40 local functions would not fit);
    // SC: the scalar operator's (p+1)^2 local functions
    constexpr int NL = SC ? (P + 1) * (P + 1) : 2 * P * (P + 1), LT = (NL + 15) / 16;
    constexpr int NB = (SC ? 2 * P * (P + 1) : NL) > 24 ? 16 : 32;
    __shared__ double sPa[NB][NL][4];
    __shared__ double sPb[NB][NL][4];
    __shared__ double2 sK[NB];
    __shared__ double sX[NB][3];
    const SingularPair sp = list[blockIdx.x];
    const int lane = threadIdx.x, half = lane >> 5, qi = lane & 31;
    int ja, a1, a2, jb, b1, b2;
    elem_of(o, sp.e, ja, a1, a2);
    elem_of(o, sp.f, jb, b1, b2);
    const int gs = o.gs, g4 = gs * gs * gs * gs;
    const int nsub = sp.kind == 1 ? 8 : (sp.kind == 2 ? 6 : 4);
    const int npts = nsub * g4;
    const double h4 = o.h * o.h * o.h * o.h;
    dx4 br[LT][LT], bi[LT][LT];
#pragma unroll
    for (int u = 0; u < LT; ++u)
#pragma unroll
        for (int v = 0; v < LT; ++v) {
            br[u][v] = dx4{0.0, 0.0, 0.0, 0.0};
            bi[u][v] = dx4{0.0, 0.0, 0.0, 0.0};
        }
    const int c = lane >> 4, m = lane & 15;
    for (int p0 = 0; p0 < npts; p0 += NB) {
        const int pt = p0 + qi;
        double X[3] = {0.0, 0.0, 0.0}, wt = 0.0;
        __syncthreads();   // the previous batch has been consumed
        if (pt < npts && qi < NB) {
            double s1, s2, t1, t2;
            singular_point(o, sp.kind, pt, s1, s2, t1, t2, wt);
            double xa, ya, xb, yb;
            if (sp.kind == 1) {
                xa = s1; ya = s2; xb = t1; yb = t2;
            } else {
                frame_map(sp.fa, s1, s2, xa, ya);
                frame_map(sp.fb, t1, t2, xb, yb);
            }
            double Fu[3], Fv[3];
            if (half == 0) {
                geom_eval(o.geo, ja, (a1 + xa) * o.h, (a2 + ya) * o.h, X, Fu, Fv);
                local_values_lds_t<P, SC>(o, a1, a2, xa, ya, Fu, Fv, o.cdiv, sPa[qi]);
            } else {
                geom_eval(o.geo, jb, (b1 + xb) * o.h, (b2 + yb) * o.h, X, Fu, Fv);
                local_values_lds_t<P, SC>(o, b1, b2, xb, yb, Fu, Fv, 1.0, sPb[qi]);
                sX[qi][0] = X[0];
                sX[qi][1] = X[1];
                sX[qi][2] = X[2];
            }
        }
        __syncthreads();
        if (half == 0 && qi < NB) {
            double2 K = make_double2(0.0, 0.0);
            if (pt < npts) {
                const double d0 = X[0] - sX[qi][0], d1 = X[1] - sX[qi][1], d2 = X[2] - sX[qi][2];
                K = cscale(wt * h4, dm::helmholtz_r2(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2))));
            }
            sK[qi] = K;
        }
        __syncthreads();
        const int nb = min(NB, npts - p0);
        for (int q = 0; q < nb; ++q) {
            const double2 K = sK[q];
            double av[LT], bv[LT];
#pragma unroll
            for (int u = 0; u < LT; ++u) {
                const int l = 16 * u + m;
                av[u] = l < NL ? sPa[q][l][c] : 0.0;
                bv[u] = l < NL ? sPb[q][l][c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < LT; ++u)
#pragma unroll
                for (int v = 0; v < LT; ++v) {
                    br[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(K.x * av[u], bv[v], br[u][v], 0, 0, 0);
                    bi[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(K.y * av[u], bv[v], bi[u][v], 0, 0, 0);
                }
        }
    }
    // lane holds B[16 u + lane/16 + 4 j][16 v + lane % 16]; the element-pair block goes
    // to its own slot, added to the near-field block by k_near_regular in list order
    double2 *dst = o.sblk + (size_t)blockIdx.x * NL * NL;
#pragma unroll
    for (int u = 0; u < LT; ++u)
#pragma unroll
        for (int v = 0; v < LT; ++v)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int l = 16 * u + (lane >> 4) + 4 * j, lb = 16 * v + (lane & 15);
                if (l < NL && lb < NL) dst[l * NL + lb] = make_double2(br[u][v][j], bi[u][v][j]);
            }
}

// ---------------------------------------------------------------------------
// a3: P2M on the leaf clusters, fused with the gather of the glued coefficients
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_p2m(DevOp o, const double2 *x, double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;            // leaf id
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen;
    const int j = id / (SL * SL), r = id % (SL * SL), k2 = r / SL, k1 = r % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    const int w1a = s + p, w2a = s + p - 1;   // component 0 block: [w2a][w1a]
    const int w1b = s + p - 1, w2b = s + p;   // component 1 block: [w2b][w1b]
    double2 *X1 = sm2;                        // [w2a][w1a]
    double2 *X2 = X1 + w2a * w1a;             // [w2b][w1b]
    double2 *Z1 = X2 + w2b * w1b;             // [w2a][Q1]
    double2 *Zd = Z1 + w2a * Q1;              // [w2a][Q1]
    double2 *Z2 = Zd + w2a * Q1;              // [w2b][Q1]
    for (int i = threadIdx.x; i < w2a * w1a; i += blockDim.x) {
        const int i2 = i / w1a, i1 = i % w1a;
        const size_t off = (((size_t)j * 2 + 0) * o.nb + (k2 * s + i2)) * o.nb + (k1 * s + i1);
        const double2 v = x[o.dof[off]];
        X1[i] = cscale((double)o.sgn[off], v);
    }
    for (int i = threadIdx.x; i < w2b * w1b; i += blockDim.x) {
        const int i2 = i / w1b, i1 = i % w1b;
        const size_t off = (((size_t)j * 2 + 1) * o.nb + (k2 * s + i2)) * o.nb + (k1 * s + i1);
        const double2 v = x[o.dof[off]];
        X2[i] = cscale((double)o.sgn[off], v);
    }
    __syncthreads();
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mqu = o.Mq + (size_t)k1 * Q1 * RL, *Mdu = o.Mdp + (size_t)k1 * Q1 * RL;
    const double *Mpv = o.Mp + (size_t)k2 * Q1 * RL, *Mqv = o.Mq + (size_t)k2 * Q1 * RL, *Mdv = o.Mdp + (size_t)k2 * Q1 * RL;
    // contract along u
    for (int i = threadIdx.x; i < w2a * Q1; i += blockDim.x) {
        const int i2 = i / Q1, m1 = i % Q1;
        double2 z = make_double2(0, 0), zd = make_double2(0, 0);
        for (int i1 = 0; i1 < w1a; ++i1) {
            const double2 v = X1[i2 * w1a + i1];
            z = cadd(z, cscale(Mpu[m1 * RL + i1], v));
            zd = cadd(zd, cscale(Mdu[m1 * RL + i1], v));
        }
        Z1[i] = z;
        Zd[i] = zd;
    }
    for (int i = threadIdx.x; i < w2b * Q1; i += blockDim.x) {
        const int i2 = i / Q1, m1 = i % Q1;
        double2 z = make_double2(0, 0);
        for (int i1 = 0; i1 < w1b; ++i1) z = cadd(z, cscale(Mqu[m1 * RL + i1], X2[i2 * w1b + i1]));
        Z2[i] = z;
    }
    __syncthreads();
    // contract along v; cartesian source vectors
    for (int mm = threadIdx.x; mm < Q; mm += blockDim.x) {
        const int m2 = mm / Q1, m1 = mm % Q1;
        double2 s1 = make_double2(0, 0), s2v = make_double2(0, 0), d = make_double2(0, 0);
        for (int i2 = 0; i2 < w2a; ++i2) {
            s1 = cadd(s1, cscale(Mqv[m2 * RL + i2], Z1[i2 * Q1 + m1]));
            d = cadd(d, cscale(Mqv[m2 * RL + i2], Zd[i2 * Q1 + m1]));
        }
        for (int i2 = 0; i2 < w2b; ++i2) {
            s2v = cadd(s2v, cscale(Mpv[m2 * RL + i2], Z2[i2 * Q1 + m1]));
            d = cadd(d, cscale(Mdv[m2 * RL + i2], Z2[i2 * Q1 + m1]));
        }
        double2 *M = mom + (size_t)gc * 3 * Q;
        M[mm] = s1;
        M[Q + mm] = s2v;
        M[2 * Q + mm] = d;
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        double2 *S = src + (size_t)gc * 4 * Q;
        for (int k = 0; k < 3; ++k) S[k * Q + mm] = cadd(cscale(T[k * Q + mm], s1), cscale(T[(3 + k) * Q + mm], s2v));
        S[3 * Q + mm] = d;
    }
}

// scalar single layer: leaf moments d = (M_p (x) M_p) c of the tensor B-spline
// coefficients over the leaf's W x W window (fields 0 and 1 stay zero), and the source
// values |J(x_m)| d at the nodes
__global__ __launch_bounds__(256) void k_p2m_sc(DevOp o, const double2 *x, double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen, W = s + p;
    const int j = id / (SL * SL), r = id % (SL * SL), k2 = r / SL, k1 = r % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    double2 *X = sm2;           // [W (i2)][W (i1)]
    double2 *Z = X + W * W;     // [W (i2)][Q1 (m1)]
    for (int i = threadIdx.x; i < W * W; i += blockDim.x) {
        const int i2 = i / W, i1 = i % W;
        X[i] = x[o.dof[((size_t)j * 2 * o.nb + (k2 * s + i2)) * o.nb + (k1 * s + i1)]];
    }
    __syncthreads();
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mpv = o.Mp + (size_t)k2 * Q1 * RL;
    for (int i = threadIdx.x; i < W * Q1; i += blockDim.x) {
        const int i2 = i / Q1, m1 = i % Q1;
        double2 z = make_double2(0, 0);
        for (int i1 = 0; i1 < W; ++i1) z = cadd(z, cscale(Mpu[m1 * RL + i1], X[i2 * W + i1]));
        Z[i] = z;
    }
    __syncthreads();
    for (int mm = threadIdx.x; mm < Q; mm += blockDim.x) {
        const int m2 = mm / Q1, m1 = mm % Q1;
        double2 d = make_double2(0, 0);
        for (int i2 = 0; i2 < W; ++i2) d = cadd(d, cscale(Mpv[m2 * RL + i2], Z[i2 * Q1 + m1]));
        double2 *M = mom + (size_t)gc * 3 * Q;
        M[mm] = make_double2(0, 0);
        M[Q + mm] = make_double2(0, 0);
        M[2 * Q + mm] = d;
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        const double Fu[3] = {T[mm], T[Q + mm], T[2 * Q + mm]}, Fv[3] = {T[3 * Q + mm], T[4 * Q + mm], T[5 * Q + mm]};
        double2 *S = src + (size_t)gc * 4 * Q;
        for (int k = 0; k < 3; ++k) S[k * Q + mm] = make_double2(0, 0);
        S[3 * Q + mm] = cscale(surf_elem(Fu, Fv), d);
    }
}

// ---------------------------------------------------------------------------
// a4: M2M, parents on level lvl from children on lvl+1
// parent[m2][m1] = sum_c sum_{n1,n2} T_c1[n1][m1] T_c2[n2][m2] child_c[n2][n1]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_m2m(DevOp o, int lvl, double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int S = 1 << lvl, Q1 = o.Q1, Q = o.Q;
    const int j = id / (S * S), r = id % (S * S), k2 = r / S, k1 = r % S;
    const int gc = (int)o.lvl_off[lvl] + id;
    double2 *ch = sm2;            // [4 children][3 fields][Q]
    double2 *W = ch + 12 * Q;     // [4][3][Q1 (n2)][Q1 (m1)]
    // one read phase: the moments of the four children
    for (int i = threadIdx.x; i < 12 * Q; i += blockDim.x) {
        const int c = i / (3 * Q), rem = i % (3 * Q);
        const int c1 = c & 1, c2 = c >> 1;
        const int cgc = (int)o.lvl_off[lvl + 1] + (j * 2 * S + 2 * k2 + c2) * 2 * S + 2 * k1 + c1;
        ch[i] = mom[(size_t)cgc * 3 * Q + rem];
    }
    __syncthreads();
    // contract along u: W[c][f][n2][m1] = sum_n1 T_c1[n1][m1] child_c[f][n2][n1]
    for (int i = threadIdx.x; i < 12 * Q; i += blockDim.x) {
        const int c = i / (3 * Q), rem = i % (3 * Q), f = rem / Q, nm = rem % Q, n2 = nm / Q1, m1 = nm % Q1;
        const double *Tu = (c & 1) ? o.T1 : o.T0;
        const double2 *cf = ch + (size_t)(c * 3 + f) * Q + n2 * Q1;
        double2 z = make_double2(0, 0);
        for (int n1 = 0; n1 < Q1; ++n1) z = cadd(z, cscale(Tu[n1 * Q1 + m1], cf[n1]));
        W[i] = z;
    }
    __syncthreads();
    // contract along v and sum the children: parent[f][m2][m1]
    for (int i = threadIdx.x; i < 3 * Q; i += blockDim.x) {
        const int f = i / Q, mm = i % Q, m2 = mm / Q1, m1 = mm % Q1;
        double2 z = make_double2(0, 0);
        for (int c = 0; c < 4; ++c) {
            const double *Tv = (c >> 1) ? o.T1 : o.T0;
            const double2 *wf = W + (size_t)(c * 3 + f) * Q;
            for (int n2 = 0; n2 < Q1; ++n2) z = cadd(z, cscale(Tv[n2 * Q1 + m2], wf[n2 * Q1 + m1]));
        }
        ch[i] = z;   // children no longer needed
    }
    __syncthreads();
    for (int mm = threadIdx.x; mm < Q; mm += blockDim.x) {
        double2 *M = mom + (size_t)gc * 3 * Q;
        const double2 s1 = ch[mm], s2v = ch[Q + mm], d = ch[2 * Q + mm];
        M[mm] = s1;
        M[Q + mm] = s2v;
        M[2 * Q + mm] = d;
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        double2 *Sv = src + (size_t)gc * 4 * Q;
        for (int k = 0; k < 3; ++k) Sv[k * Q + mm] = cadd(cscale(T[k * Q + mm], s1), cscale(T[(3 + k) * Q + mm], s2v));
        if (o.scalar) {   // scalar: the moments times the surface element at the node
            const double Fu[3] = {T[mm], T[Q + mm], T[2 * Q + mm]}, Fv[3] = {T[3 * Q + mm], T[4 * Q + mm], T[5 * Q + mm]};
            Sv[3 * Q + mm] = cscale(surf_elem(Fu, Fv), d);
        } else {
            Sv[3 * Q + mm] = d;
        }
    }
}

// Levels of a smaller interpolation degree q_l (variable order): their moments are the
// exact restriction of the degree-q moments, m_l = (R_l (x) R_l)^T m with
// R_l[n][m] = L^{q_l}_m(x^q_n), turned into the source fields at the level's own nodes;
// the coupling's local expansions go back through R_l (x) R_l before L2L.
__global__ __launch_bounds__(256) void k_restrict(DevOp o, int lvl, const double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int gc = (int)o.lvl_off[lvl] + blockIdx.x;
    const int Q1h = o.Q1, Qs = o.Q, Q1l = o.ql[lvl] + 1, Ql = Q1l * Q1l;
    const double *R = o.Rl + (size_t)lvl * Q1h * Q1h;   // [n][m], m < Q1l
    double2 *M = sm2;               // [3][Qs]
    double2 *Z = M + 3 * Qs;        // [3][Q1h (n2)][Q1l (m1)]
    for (int i = threadIdx.x; i < 3 * Qs; i += blockDim.x) M[i] = mom[(size_t)gc * 3 * Qs + i];
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Q1h * Q1l; i += blockDim.x) {
        const int f = i / (Q1h * Q1l), r = i % (Q1h * Q1l), n2 = r / Q1l, m1 = r % Q1l;
        double2 z = make_double2(0, 0);
        for (int n1 = 0; n1 < Q1h; ++n1) z = cadd(z, cscale(R[n1 * Q1h + m1], M[f * Qs + n2 * Q1h + n1]));
        Z[i] = z;
    }
    __syncthreads();
    const double *T = o.nodeT + (size_t)gc * 6 * Qs;
    double2 *Sv = src + (size_t)gc * 4 * Qs;
    for (int mm = threadIdx.x; mm < Ql; mm += blockDim.x) {
        const int m2 = mm / Q1l, m1 = mm % Q1l;
        double2 sf[3];
        for (int f = 0; f < 3; ++f) {
            double2 v = make_double2(0, 0);
            for (int n2 = 0; n2 < Q1h; ++n2) v = cadd(v, cscale(R[n2 * Q1h + m2], Z[(f * Q1h + n2) * Q1l + m1]));
            sf[f] = v;
        }
        const double Fu[3] = {T[mm], T[Qs + mm], T[2 * Qs + mm]}, Fv[3] = {T[3 * Qs + mm], T[4 * Qs + mm], T[5 * Qs + mm]};
        if (o.scalar) {
            for (int k = 0; k < 3; ++k) Sv[k * Qs + mm] = make_double2(0, 0);
            Sv[3 * Qs + mm] = cscale(surf_elem(Fu, Fv), sf[2]);
        } else {
            for (int k = 0; k < 3; ++k) Sv[k * Qs + mm] = cadd(cscale(Fu[k], sf[0]), cscale(Fv[k], sf[1]));
            Sv[3 * Qs + mm] = sf[2];
        }
    }
}

__global__ __launch_bounds__(256) void k_lift(DevOp o, int lvl, double2 *loc)
{
    extern __shared__ double2 sm2[];
    const int gc = (int)o.lvl_off[lvl] + blockIdx.x;
    const int Q1h = o.Q1, Qs = o.Q, Q1l = o.ql[lvl] + 1, Ql = Q1l * Q1l;
    const double *R = o.Rl + (size_t)lvl * Q1h * Q1h;
    double2 *A = sm2;               // [3][Ql]
    double2 *Y = A + 3 * Ql;        // [3][Q1l (m2)][Q1h (n1)]
    double2 *Lc = loc + (size_t)gc * 3 * Qs;
    for (int i = threadIdx.x; i < 3 * Ql; i += blockDim.x) A[i] = Lc[(i / Ql) * Qs + i % Ql];
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Q1l * Q1h; i += blockDim.x) {
        const int f = i / (Q1l * Q1h), r = i % (Q1l * Q1h), m2 = r / Q1h, n1 = r % Q1h;
        double2 y = make_double2(0, 0);
        for (int m1 = 0; m1 < Q1l; ++m1) y = cadd(y, cscale(R[n1 * Q1h + m1], A[f * Ql + m2 * Q1l + m1]));
        Y[i] = y;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Qs; i += blockDim.x) {
        const int f = i / Qs, nn = i % Qs, n2 = nn / Q1h, n1 = nn % Q1h;
        double2 v = make_double2(0, 0);
        for (int m2 = 0; m2 < Q1l; ++m2) v = cadd(v, cscale(R[n2 * Q1h + m2], Y[(f * Q1l + m2) * Q1h + n1]));
        Lc[i] = v;
    }
}

// ---------------------------------------------------------------------------
// a5: M2L. Work item = (target cluster, range of far partners).  The localized
// kernel is interpolated in both parameter squares:
//   u[m] += sum_m' G(|x_m - x'_m'|) (v_x, v_y, v_z, d)'[m']
// Threads: kM2LNT target nodes each (register blocking: every source value read
// from LDS serves kM2LNT targets) x a part of the source nodes; the parts are
// summed once per work item through LDS.
// ---------------------------------------------------------------------------
constexpr int kM2LThreads = 256;
constexpr int kM2LNT = 3;
constexpr int kQMaxSym = 81;    // nodes per cluster of the unordered-pair coupling (degree <= 8)

template <typename T>
__global__ __launch_bounds__(kM2LThreads) void k_m2l(DevOp o, int nwork, const M2LWork *work, const int32_t *partner,
                                                      const double2 *src, double2 *part)
{
    using C = typename dm::cplx_of<T>::type;
    extern __shared__ double smd[];
    __shared__ double2 sTab[256];                               // (cos, sin)(j pi/128) / (4 pi), FP64 only
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < 256; i += kM2LThreads) sTab[i] = o.sctab[i];   // first use after a barrier
    // one work item per workgroup, or (a grid smaller than the work) items blockIdx.x,
    // blockIdx.x + gridDim.x, ...
    for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const M2LWork wk = work[wi];
    // nodes of the target's level (the partners are on the same level); per-cluster
    // arrays keep the stride Qs of the largest degree
    const int Qs = o.Q;
    int lvw = 0;
    while (lvw < o.L && wk.tgt >= o.lvl_off[lvw + 1]) ++lvw;
    const int Q = (o.ql[lvw] + 1) * (o.ql[lvw] + 1);
    const int TPG = (Q + kM2LNT - 1) / kM2LNT;
    const int S = min(kM2LThreads / TPG, Q);
    const int SP = (Q + S - 1) / S;
    const int tid = threadIdx.x;
    const int mt = tid % TPG, sp = tid / TPG;
    const bool active = sp < S;
    // node-major staging, so one address (and immediate offsets) reaches a node's data
    T *sX = reinterpret_cast<T *>(smd);                        // [Q][4]: x, y, z, unused
    C *sV = reinterpret_cast<C *>(smd + (4 * Q * (int)sizeof(T) + 15) / 16 * 2);   // [Q][4], 16-B aligned after sX
    double2 *red = reinterpret_cast<double2 *>(smd);           // [S][Q][2] after the partner loop
    const T kap = (T)o.kappa;
    T xt[kM2LNT][3];
    bool val[kM2LNT];
    C acc[kM2LNT][4];
    const double *Xt = o.nodeX + (size_t)wk.tgt * 3 * Qs;
#pragma unroll
    for (int k = 0; k < kM2LNT; ++k) {
        const int mm = mt + k * TPG;
        val[k] = active && mm < Q;
        const int mc = val[k] ? mm : 0;
        xt[k][0] = (T)Xt[mc];
        xt[k][1] = (T)Xt[Qs + mc];
        xt[k][2] = (T)Xt[2 * Qs + mc];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[k][j] = C{0, 0};
    }
    const int mb = min(Q, sp * SP), me = min(Q, mb + SP);
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const int sc = partner[kp];
        __syncthreads();
        const double *Xs = o.nodeX + (size_t)sc * 3 * Qs;
        const double2 *Vs = src + (size_t)sc * 4 * Qs;
        for (int i = tid; i < 3 * Q; i += kM2LThreads) sX[(i % Q) * 4 + i / Q] = (T)Xs[(i / Q) * Qs + i % Q];
        for (int i = tid; i < 4 * Q; i += kM2LThreads) sV[(i % Q) * 4 + i / Q] = dm::to_c(Vs[(i / Q) * Qs + i % Q], T(0));
        __syncthreads();
        if (active) {
            for (int ms = mb; ms < me; ++ms) {
                const T x0 = sX[4 * ms], x1 = sX[4 * ms + 1], x2 = sX[4 * ms + 2];
                const C v0 = sV[4 * ms], v1 = sV[4 * ms + 1], v2 = sV[4 * ms + 2], v3 = sV[4 * ms + 3];
#pragma unroll
                for (int k = 0; k < kM2LNT; ++k) {
                    const T d0 = xt[k][0] - x0, d1 = xt[k][1] - x1, d2 = xt[k][2] - x2;
                    C G;
                    if constexpr (sizeof(T) == 8) G = dm::helmholtz_r2_tab(kap, fma(d0, d0, fma(d1, d1, d2 * d2)), sTab);
                    else G = dm::helmholtz_r2(kap, fma(d0, d0, fma(d1, d1, d2 * d2)));
                    acc[k][0] = dm::cmac(acc[k][0], G, v0);
                    acc[k][1] = dm::cmac(acc[k][1], G, v1);
                    acc[k][2] = dm::cmac(acc[k][2], G, v2);
                    acc[k][3] = dm::cmac(acc[k][3], G, v3);
                }
            }
        }
    }
    // the source parts summed in a fixed order, two fields at a time (half the
    // shared memory of all four: one more workgroup per CU)
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kM2LNT; ++k)
            if (val[k]) {
                const int mm = mt + k * TPG;
#pragma unroll
                for (int j = 0; j < 2; ++j) red[((size_t)sp * Q + mm) * 2 + j] = dm::to_d(acc[k][2 * hf + j]);
            }
        __syncthreads();
        for (int i = tid; i < 2 * Q; i += kM2LThreads) {
            const int j = i / Q, mm = i % Q;
            double2 v = make_double2(0, 0);
            for (int q2 = 0; q2 < S; ++q2) v = cadd(v, red[((size_t)q2 * Q + mm) * 2 + j]);
            part[((size_t)wi * 4 + 2 * hf + j) * Qs + mm] = v;
        }
    }
    __syncthreads();   // the next item's staging reuses the shared memory
    }
}

// ---------------------------------------------------------------------------
// a5 over unordered pairs (one FP64 column, one degree on every level).  The kernel
// is symmetric, G(x, y) = G(y, x), and both clusters of a far pair sit on one level
// with the same reference nodes, so the block of (s, t) is the transpose of the
// block of (t, s).  Work item = cluster t with a chunk of partners s > t; every
// kernel value is evaluated once and serves both sides:
//   u_t[m]  += sum_m' G(|x_m - x'_m'|) v_s[m']   (row side, summed over the chunk)
//   u_s[m'] += sum_m  G(|x_m - x'_m'|) v_t[m]    (column side, per pair)
// Rows are taken in kM2LNT chunks of TPG rows.  In the row layout a thread holds
// one row of the chunk and a range of columns (the row side accumulates in
// registers); the chunk's values go to shared memory, and in the column layout a
// thread holds kM2LNT columns and a range of the chunk's rows.  The column side's
// parts are summed in a fixed order once per pair, the row side's once per item.
// Slots of part: item i -> i (row side), partner k -> nwork + k (column side).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kM2LThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_m2l_sym(
    DevOp o, int nwork, const M2LWork *work, const int32_t *partner, const double2 *src, double2 *part)
{
    extern __shared__ double smd[];
    __shared__ double2 sTab[256];                               // (cos, sin)(j pi/128) / (4 pi)
    for (int i = threadIdx.x; i < 256; i += kM2LThreads) sTab[i] = o.sctab[i];   // first use after a barrier
    const M2LWork wk = work[blockIdx.x];
    const int Q = o.Q;
    const int TPG = (Q + kM2LNT - 1) / kM2LNT;
    const int S = min(kM2LThreads / TPG, Q);
    const int SP = (Q + S - 1) / S;       // columns per thread (row layout)
    const int RP = (TPG + S - 1) / S;     // chunk rows per thread (column layout)
    const int tid = threadIdx.x;
    const int mt = tid % TPG, sp = tid / TPG;
    const bool active = sp < S;
    double *sX = smd;                                            // [Q][4] partner's nodes
    double2 *sV = reinterpret_cast<double2 *>(smd + 4 * Q);     // [Q][4] partner's source fields
    double2 *sW = sV + 4 * Q;                                    // [Q][4] row cluster's source fields
    double2 *sG = sW + 4 * Q;                                    // [Q][TPG] chunk of G, column-major
    double2 *red = sG;                                           // [S][Q][2] reductions
    const double kap = o.kappa;
    double xt[kM2LNT][3];
    bool val[kM2LNT];
    double2 acc[kM2LNT][4], cac[kM2LNT][4];
    const double *Xt = o.nodeX + (size_t)wk.tgt * 3 * Q;
#pragma unroll
    for (int k = 0; k < kM2LNT; ++k) {
        const int mm = mt + k * TPG;
        val[k] = active && mm < Q;
        const int mc = val[k] ? mm : 0;
        xt[k][0] = Xt[mc];
        xt[k][1] = Xt[Q + mc];
        xt[k][2] = Xt[2 * Q + mc];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[k][j] = make_double2(0, 0);
    }
    {
        const double2 *Vt = src + (size_t)wk.tgt * 4 * Q;
        for (int i = tid; i < 4 * Q; i += kM2LThreads) sW[(i % Q) * 4 + i / Q] = Vt[i];
    }
    const int mb = min(Q, sp * SP), me = min(Q, mb + SP);
    const int rb = sp * RP, re = min(TPG, rb + RP);
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const int sc = partner[kp];
        __syncthreads();
        const double *Xs = o.nodeX + (size_t)sc * 3 * Q;
        const double2 *Vs = src + (size_t)sc * 4 * Q;
        for (int i = tid; i < 3 * Q; i += kM2LThreads) sX[(i % Q) * 4 + i / Q] = Xs[i];
        for (int i = tid; i < 4 * Q; i += kM2LThreads) sV[(i % Q) * 4 + i / Q] = Vs[i];
#pragma unroll
        for (int k = 0; k < kM2LNT; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) cac[k][j] = make_double2(0, 0);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kM2LNT; ++c) {
            if (c * TPG >= Q) break;   // uniform
            // row layout: row c TPG + mt against the columns [mb, me)
            if (val[c]) {
                for (int ms = mb; ms < me; ++ms) {
                    const double d0 = xt[c][0] - sX[4 * ms], d1 = xt[c][1] - sX[4 * ms + 1], d2 = xt[c][2] - sX[4 * ms + 2];
                    const double2 G = dm::helmholtz_r2_tab(kap, fma(d0, d0, fma(d1, d1, d2 * d2)), sTab);
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[c][j] = dm::cmac(acc[c][j], G, sV[4 * ms + j]);
                    sG[ms * TPG + mt] = G;
                }
            }
            __syncthreads();
            // column layout: columns mt + k TPG against the chunk rows [rb, re)
            if (active) {
                for (int r = rb; r < re; ++r) {
                    const int gr = c * TPG + r;
                    if (gr >= Q) break;
                    const double2 w0 = sW[4 * gr], w1 = sW[4 * gr + 1], w2 = sW[4 * gr + 2], w3 = sW[4 * gr + 3];
#pragma unroll
                    for (int k = 0; k < kM2LNT; ++k)
                        if (val[k]) {
                            const double2 G = sG[(mt + k * TPG) * TPG + r];
                            cac[k][0] = dm::cmac(cac[k][0], G, w0);
                            cac[k][1] = dm::cmac(cac[k][1], G, w1);
                            cac[k][2] = dm::cmac(cac[k][2], G, w2);
                            cac[k][3] = dm::cmac(cac[k][3], G, w3);
                        }
                }
            }
            __syncthreads();
        }
        // column side of the pair: the S row ranges summed in order, two fields at a time
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
            for (int k = 0; k < kM2LNT; ++k)
                if (val[k]) {
                    const int mm = mt + k * TPG;
#pragma unroll
                    for (int j = 0; j < 2; ++j) red[((size_t)sp * Q + mm) * 2 + j] = cac[k][2 * hf + j];
                }
            __syncthreads();
            for (int i = tid; i < 2 * Q; i += kM2LThreads) {
                const int j = i / Q, mm = i % Q;
                double2 v = make_double2(0, 0);
                for (int q2 = 0; q2 < S; ++q2) v = cadd(v, red[((size_t)q2 * Q + mm) * 2 + j]);
                part[((size_t)(nwork + kp) * 4 + 2 * hf + j) * Q + mm] = v;
            }
            __syncthreads();
        }
    }
    // row side: the column ranges summed in order, two fields at a time
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kM2LNT; ++k)
            if (val[k]) {
                const int mm = mt + k * TPG;
#pragma unroll
                for (int j = 0; j < 2; ++j) red[((size_t)sp * Q + mm) * 2 + j] = acc[k][2 * hf + j];
            }
        __syncthreads();
        for (int i = tid; i < 2 * Q; i += kM2LThreads) {
            const int j = i / Q, mm = i % Q;
            double2 v = make_double2(0, 0);
            for (int q2 = 0; q2 < S; ++q2) v = cadd(v, red[((size_t)q2 * Q + mm) * 2 + j]);
            part[((size_t)blockIdx.x * 4 + 2 * hf + j) * Q + mm] = v;
        }
    }
}

// per cluster, the sum of its slots in list order (row sides of its items, then the
// column sides of its pairs), converted to the test-side fields as below
// (loads issued eight slots at a time, added in list order)
__global__ __launch_bounds__(512) void k_m2l_reduce_sym(DevOp o, const int32_t *ptr, const int32_t *idx,
                                                        const double2 *part, double2 *loc)
{
    __shared__ double2 su[4][kQMaxSym];
    const int gc = blockIdx.x, Q = o.Q;
    const int b = ptr[gc], e = ptr[gc + 1];
    for (int i = threadIdx.x; i < 4 * Q; i += blockDim.x) {
        double2 v = make_double2(0, 0);
        for (int w0 = b; w0 < e; w0 += 8) {
            double2 t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                t[u] = w0 + u < e ? part[(size_t)idx[w0 + u] * 4 * Q + i] : make_double2(0, 0);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (w0 + u < e) v = cadd(v, t[u]);
        }
        su[i / Q][i % Q] = v;
    }
    __syncthreads();
    const double ik2 = 1.0 / (o.kappa * o.kappa);
    for (int mm = threadIdx.x; mm < Q; mm += blockDim.x) {
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        double2 *L = loc + (size_t)gc * 3 * Q;
        if (o.scalar) {   // scalar: t = |J(x_m)| u (the target's surface element)
            const double Fu[3] = {T[mm], T[Q + mm], T[2 * Q + mm]}, Fv[3] = {T[3 * Q + mm], T[4 * Q + mm], T[5 * Q + mm]};
            L[mm] = make_double2(0, 0);
            L[Q + mm] = make_double2(0, 0);
            L[2 * Q + mm] = cscale(surf_elem(Fu, Fv), su[3][mm]);
            continue;
        }
        double2 t1 = make_double2(0, 0), t2 = make_double2(0, 0);
        for (int k = 0; k < 3; ++k) {
            t1 = cadd(t1, cscale(T[k * Q + mm], su[k][mm]));
            t2 = cadd(t2, cscale(T[(3 + k) * Q + mm], su[k][mm]));
        }
        L[mm] = t1;
        L[Q + mm] = t2;
        L[2 * Q + mm] = cscale(-ik2, su[3][mm]);
    }
}

// sum the partial couplings of every cluster (fixed order) and convert to the
// test-side fields t^a = d_aF . u_xyz, t^d = -kappa^-2 u_d
__global__ void k_m2l_reduce(DevOp o, const int32_t *wrk_of_tgt, const double2 *part, double2 *loc)
{
    const int gc = blockIdx.x, Qs = o.Q;
    int lvl = 0;
    while (lvl < o.L && gc >= o.lvl_off[lvl + 1]) ++lvl;
    const int Q = (o.ql[lvl] + 1) * (o.ql[lvl] + 1);   // nodes of the level (stride Qs)
    const int b = wrk_of_tgt[gc], e = wrk_of_tgt[gc + 1];
    const double ik2 = 1.0 / (o.kappa * o.kappa);
    for (int mm = threadIdx.x; mm < Q; mm += blockDim.x) {
        double2 u[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
        for (int w = b; w < e; ++w)
            for (int k = 0; k < 4; ++k) u[k] = cadd(u[k], part[((size_t)w * 4 + k) * Qs + mm]);
        const double *T = o.nodeT + (size_t)gc * 6 * Qs;
        double2 t1 = make_double2(0, 0), t2 = make_double2(0, 0);
        for (int k = 0; k < 3; ++k) {
            t1 = cadd(t1, cscale(T[k * Qs + mm], u[k]));
            t2 = cadd(t2, cscale(T[(3 + k) * Qs + mm], u[k]));
        }
        double2 *L = loc + (size_t)gc * 3 * Qs;
        if (o.scalar) {   // scalar: t = |J(x_m)| u (the localized kernel's target surface element)
            const double Fu[3] = {T[mm], T[Qs + mm], T[2 * Qs + mm]}, Fv[3] = {T[3 * Qs + mm], T[4 * Qs + mm], T[5 * Qs + mm]};
            L[mm] = make_double2(0, 0);
            L[Qs + mm] = make_double2(0, 0);
            L[2 * Qs + mm] = cscale(surf_elem(Fu, Fv), u[3]);
            continue;
        }
        L[mm] = t1;
        L[Qs + mm] = t2;
        L[2 * Qs + mm] = cscale(-ik2, u[3]);
    }
}

// ---------------------------------------------------------------------------
// a6: L2L, children on level lvl from parents on lvl-1
// child[n2][n1] += sum_{m1,m2} T_c1[n1][m1] T_c2[n2][m2] parent[m2][m1]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_l2l(DevOp o, int lvl, double2 *loc)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int S = 1 << lvl, Q1 = o.Q1, Q = o.Q;
    const int j = id / (S * S), r = id % (S * S), k2 = r / S, k1 = r % S;
    const int gc = (int)o.lvl_off[lvl] + id;
    const int Sp = S / 2;
    const int pgc = (int)o.lvl_off[lvl - 1] + (j * Sp + k2 / 2) * Sp + k1 / 2;
    const int c1 = k1 & 1, c2 = k2 & 1;
    const double *Tu = c1 ? o.T1 : o.T0, *Tv = c2 ? o.T1 : o.T0;
    const double2 *par = loc + (size_t)pgc * 3 * Q;
    double2 *W = sm2;   // [3][Q1 (m2)][Q1 (n1)]
    for (int i = threadIdx.x; i < 3 * Q; i += blockDim.x) {
        const int f = i / Q, rem = i % Q, m2 = rem / Q1, n1 = rem % Q1;
        double2 z = make_double2(0, 0);
        for (int m1 = 0; m1 < Q1; ++m1) z = cadd(z, cscale(Tu[n1 * Q1 + m1], par[f * Q + m2 * Q1 + m1]));
        W[i] = z;
    }
    __syncthreads();
    double2 *ch = loc + (size_t)gc * 3 * Q;
    for (int i = threadIdx.x; i < 3 * Q; i += blockDim.x) {
        const int f = i / Q, rem = i % Q, n2 = rem / Q1, n1 = rem % Q1;
        double2 z = ch[i];
        for (int m2 = 0; m2 < Q1; ++m2) z = cadd(z, cscale(Tv[n2 * Q1 + m2], W[f * Q + m2 * Q1 + n1]));
        ch[i] = z;
    }
}

// ---------------------------------------------------------------------------
// a8: near-field product.  A workgroup streams rc rows of one stored block B
// (target leaf t, source leaf s) once: every row gives the row partial
// (B x_s)[k] and, for t != s, the same loads give the column partials of B^T x_t
// over the chunk.  Lanes own columns (coalesced 16-byte loads, bypassing the
// caches); the four waves take every fourth row and combine their column
// partials in a fixed order.
// ---------------------------------------------------------------------------
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline d2v ld_blk(const double2 *B, size_t i)
{
    return __builtin_nontemporal_load(reinterpret_cast<const d2v *>(B) + i);
}

template <int U>
__global__ __launch_bounds__(256) void k_near_blk(DevOp o, const double2 *x, double2 *part)
{
    __shared__ double2 sxr[64 * U];
    __shared__ double2 syc[3][64 * U];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.x / o.nch;
    const int ch = blockIdx.x % o.nch;
    const int lt = o.bpair[2 * b], ls = o.bpair[2 * b + 1];
    const int nF = o.nF, r0 = ch * o.rc, r1 = min(nF, r0 + o.rc);
    d2v xc[U], yc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int c = lane + 64 * u;
        const int d = c < nF ? o.leafdof[(size_t)ls * nF + c] : -1;
        const double2 v = d >= 0 ? x[d] : make_double2(0.0, 0.0);
        xc[u] = d2v{v.x, v.y};
        yc[u] = d2v{0.0, 0.0};
    }
    for (int k = threadIdx.x; k < r1 - r0; k += blockDim.x) {
        const int d = o.leafdof[(size_t)lt * nF + r0 + k];
        sxr[k] = d >= 0 ? x[d] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const double2 *B = o.bval + (size_t)b * nF * nF;
    int r = r0 + wv;
    // RS rows per step (r, r + 4, ...): RS U independent streaming loads in flight per
    // lane; the last step of a wave may hold fewer rows (the others load and add zeros)
    constexpr int RS = 2;
    for (; r < r1; r += 4 * RS) {
        d2v al[RS][U];
#pragma unroll
        for (int q = 0; q < RS; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lane + 64 * u;
                al[q][u] = (c < nF && r + 4 * q < r1) ? ld_blk(B, (size_t)(r + 4 * q) * nF + c) : d2v{0.0, 0.0};
            }
        double2 xq[RS];
        double re[RS], im[RS];
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            xq[q] = r + 4 * q < r1 ? sxr[r + 4 * q - r0] : make_double2(0.0, 0.0);
            re[q] = 0.0;
            im[q] = 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            d2v a[RS];
#pragma unroll
            for (int q = 0; q < RS; ++q) a[q] = al[q][u];
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                re[q] = fma(a[q].x, xc[u].x, fma(-a[q].y, xc[u].y, re[q]));
                im[q] = fma(a[q].x, xc[u].y, fma(a[q].y, xc[u].x, im[q]));
            }
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                yc[u].x = fma(a[q].x, xq[q].x, fma(-a[q].y, xq[q].y, yc[u].x));
                yc[u].y = fma(a[q].x, xq[q].y, fma(a[q].y, xq[q].x, yc[u].y));
            }
        }
        // the 2 RS row sums over the wave by recursive halving (one value per lane group)
        double v[2 * RS];
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            v[2 * q] = re[q];
            v[2 * q + 1] = im[q];
        }
        const double tot = dm::Halve<2 * RS>::run(v, lane, 32);
        constexpr int SH = 6 - dm::log2c<2 * RS>();
        if ((lane & ((1 << SH) - 1)) == 0) {
            const int k = lane >> SH;   // value 2 q + (0: real, 1: imaginary part)
            if (r + 4 * (k >> 1) < r1)
                reinterpret_cast<double *>(part)[2 * ((size_t)b * nF + r + 4 * (k >> 1)) + (k & 1)] = tot;
        }
    }
    if (lt == ls) return;   // diagonal block: no transposed product (uniform branch)
    if (wv > 0)
#pragma unroll
        for (int u = 0; u < U; ++u) syc[wv - 1][lane + 64 * u] = make_double2(yc[u].x, yc[u].y);
    __syncthreads();
    if (wv == 0) {
        double2 *cp = part + (size_t)o.nblk * nF + ((size_t)b * o.nch + ch) * nF;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = lane + 64 * u;
            if (c < nF) {
                const double2 s1 = syc[0][c], s2 = syc[1][c], s3 = syc[2][c];
                cp[c] = make_double2(((yc[u].x + s1.x) + s2.x) + s3.x, ((yc[u].y + s1.y) + s2.y) + s3.y);
            }
        }
    }
}

// y[i] = sum of the partial results of unknown i: 16 lanes take every 16th entry of
// its list, then a fixed butterfly (the order does not depend on the launch)
__global__ __launch_bounds__(256) void k_near_gather(int N, const int64_t *ptr, const int32_t *idx,
                                                     const double2 *part, double2 *y)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t >> 4), sub = (int)(t & 15);
    double re = 0.0, im = 0.0;
    if (i < N)
        for (int64_t k = ptr[i] + sub; k < ptr[i + 1]; k += 16) {
            const double2 v = part[idx[k]];
            re += v.x;
            im += v.y;
        }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off, 16);
        im += __shfl_xor(im, off, 16);
    }
    if (i < N && sub == 0) y[i] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// a7: L2P.  Per leaf cluster, the test-side moments of the local spline pieces
// against the local fields (tensor contraction, u then v):
//   Y0[i2][i1] = sum Mp(k1)[m1][i1] Mq(k2)[m2][i2] t^1[m2][m1] + Mdp(k1) Mq(k2) t^d
//   Y1[i2][i1] = sum Mq(k1)[m1][i1] Mp(k2)[m2][i2] t^2[m2][m1] + Mq(k1) Mdp(k2) t^d
// then one thread per unknown gathers (with the gluing sign) the entries of the
// leaf clusters that its incarnations touch: the scatter T^T without atomics.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_l2p_leaf(DevOp o, const double2 *loc, double2 *ybuf)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen;
    const int r = id % (SL * SL), k2 = r / SL, k1 = r % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    const double2 *t = loc + (size_t)gc * 3 * Q;
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mqu = o.Mq + (size_t)k1 * Q1 * RL, *Mdu = o.Mdp + (size_t)k1 * Q1 * RL;
    const double *Mpv = o.Mp + (size_t)k2 * Q1 * RL, *Mqv = o.Mq + (size_t)k2 * Q1 * RL, *Mdv = o.Mdp + (size_t)k2 * Q1 * RL;
    double2 *W0 = sm2;                 // [Q1 (m2)][RL (i1)]  component 0 field + divergence
    double2 *W1 = W0 + Q1 * RL;        // component 1 field
    double2 *W1d = W1 + Q1 * RL;       // component 1 divergence
    const int w1a = s + p, w1b = s + p - 1;
    for (int i = threadIdx.x; i < Q1 * RL; i += blockDim.x) {
        const int m2 = i / RL, i1 = i % RL;
        double2 a = make_double2(0, 0), b = make_double2(0, 0), bd = make_double2(0, 0);
        for (int m1 = 0; m1 < Q1; ++m1) {
            const double2 f1 = t[m2 * Q1 + m1], f2 = t[Q + m2 * Q1 + m1], fd = t[2 * Q + m2 * Q1 + m1];
            if (i1 < w1a) a = cadd(a, cadd(cscale(Mpu[m1 * RL + i1], f1), cscale(Mdu[m1 * RL + i1], fd)));
            if (i1 < w1b) {
                b = cadd(b, cscale(Mqu[m1 * RL + i1], f2));
                bd = cadd(bd, cscale(Mqu[m1 * RL + i1], fd));
            }
        }
        W0[i] = a;
        W1[i] = b;
        W1d[i] = bd;
    }
    __syncthreads();
    double2 *Y = ybuf + (size_t)id * 2 * RL * RL;
    for (int i = threadIdx.x; i < 2 * RL * RL; i += blockDim.x) {
        const int c = i / (RL * RL), rem = i % (RL * RL), i2 = rem / RL, i1 = rem % RL;
        double2 v = make_double2(0, 0);
        if (c == 0 && i2 < s + p - 1 && i1 < w1a) {
            for (int m2 = 0; m2 < Q1; ++m2) v = cadd(v, cscale(Mqv[m2 * RL + i2], W0[m2 * RL + i1]));
        } else if (c == 1 && i2 < s + p && i1 < w1b) {
            for (int m2 = 0; m2 < Q1; ++m2)
                v = cadd(v, cadd(cscale(Mpv[m2 * RL + i2], W1[m2 * RL + i1]), cscale(Mdv[m2 * RL + i2], W1d[m2 * RL + i1])));
        }
        Y[i] = v;
    }
}

// scalar single layer: Y[i2][i1] = sum (M_p (x) M_p)^T t^d over the leaf's W x W window
// (component 0 of the leaf's result rows)
__global__ __launch_bounds__(256) void k_l2p_leaf_sc(DevOp o, const double2 *loc, double2 *ybuf)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen, W = s + p;
    const int r = id % (SL * SL), k2 = r / SL, k1 = r % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    const double2 *t = loc + (size_t)gc * 3 * Q + 2 * Q;
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mpv = o.Mp + (size_t)k2 * Q1 * RL;
    double2 *Wm = sm2;   // [Q1 (m2)][W (i1)]
    for (int i = threadIdx.x; i < Q1 * W; i += blockDim.x) {
        const int m2 = i / W, i1 = i % W;
        double2 a = make_double2(0, 0);
        for (int m1 = 0; m1 < Q1; ++m1) a = cadd(a, cscale(Mpu[m1 * RL + i1], t[m2 * Q1 + m1]));
        Wm[i] = a;
    }
    __syncthreads();
    double2 *Y = ybuf + (size_t)id * 2 * RL * RL;
    for (int i = threadIdx.x; i < RL * RL; i += blockDim.x) {
        const int i2 = i / RL, i1 = i % RL;
        double2 v = make_double2(0, 0);
        if (i2 < W && i1 < W)
            for (int m2 = 0; m2 < Q1; ++m2) v = cadd(v, cscale(Mpv[m2 * RL + i2], Wm[m2 * W + i1]));
        Y[i] = v;
    }
}

__global__ void k_l2p_gather(DevOp o, const double2 *ybuf, double2 *y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= o.N) return;
    const int s = o.s, p = o.p, SL = o.SL, n = o.n, RL = o.rowlen;
    double2 acc = make_double2(0, 0);
    for (int c = 0; c < 2; ++c) {
        const int32_t *in = o.inc + ((size_t)i * 2 + c) * 5;
        const int j = in[0];
        if (j < 0) continue;
        const int a = in[1], i1 = in[2], i2 = in[3];
        const double sg = (double)in[4];
        const int du = (a == 0) ? p : p - 1, dv = (a == 0 && !o.scalar) ? p - 1 : p;
        const int k1b = max(0, i1 - du) / s, k1e = min(n - 1, i1) / s;
        const int k2b = max(0, i2 - dv) / s, k2e = min(n - 1, i2) / s;
        for (int k2 = k2b; k2 <= k2e; ++k2)
            for (int k1 = k1b; k1 <= k1e; ++k1) {
                const int leaf = (j * SL + k2) * SL + k1;
                const double2 v = ybuf[(((size_t)leaf * 2 + a) * RL + (i2 - k2 * s)) * RL + (i1 - k1 * s)];
                acc = cadd(acc, cscale(sg, v));
            }
    }
    y[i] = cadd(y[i], acc);
}

// ---------------------------------------------------------------------------
// a9: plane-wave right-hand side, one thread per unknown
// f_i = - sum_e sum_q e_inc(X_q) . w_q phi_hat_i d_aF
// ---------------------------------------------------------------------------
__global__ void k_rhs_plane(DevOp o, double d0, double d1, double d2, double2 p0, double2 p1, double2 p2, double2 *f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= o.N) return;
    const int p = o.p, n = o.n, G2 = o.G2, NL = o.nl;
    double2 acc = make_double2(0, 0);
    for (int c = 0; c < 2; ++c) {
        const int32_t *in = o.inc + ((size_t)i * 2 + c) * 5;
        const int j = in[0];
        if (j < 0) continue;
        const int a = in[1], i1 = in[2], i2 = in[3];
        const double sg = (double)in[4];
        const int du = (a == 0) ? p : p - 1, dv = (a == 0) ? p - 1 : p;
        for (int e2 = max(0, i2 - dv); e2 <= min(n - 1, i2); ++e2)
            for (int e1 = max(0, i1 - du); e1 <= min(n - 1, i1); ++e1) {
                const int t1 = i1 - e1, t2 = i2 - e2;
                const int l = (a == 0) ? t2 * (p + 1) + t1 : p * (p + 1) + t2 * p + t1;
                const int64_t e = ((int64_t)j * n + e2) * n + e1;
                const double *X = o.eX + e * 3 * G2;
                const double *Ps = o.ePsi + e * 4 * NL * G2;
                for (int q = 0; q < G2; ++q) {
                    const double ph = o.kappa * (d0 * X[q] + d1 * X[G2 + q] + d2 * X[2 * G2 + q]);
                    double sn, cs;
                    sincos(ph, &sn, &cs);
                    const double2 ex = make_double2(cs, sn);
                    const double f0 = Ps[((size_t)0 * NL + l) * G2 + q], f1 = Ps[((size_t)1 * NL + l) * G2 + q],
                                 f2 = Ps[((size_t)2 * NL + l) * G2 + q];
                    const double2 dotp = cadd(cadd(cscale(f0, p0), cscale(f1, p1)), cscale(f2, p2));
                    acc = cadd(acc, cscale(-sg, cmul(ex, dotp)));
                }
            }
    }
    f[i] = acc;
}

// scalar single layer right-hand side f_i = int g phi_i dsigma, one thread per unknown:
// kind 0 plane wave g = exp(i kappa a.x), kind 1 point source g = G(x - a)
__global__ void k_rhs_scalar(DevOp o, int kind, double a0, double a1, double a2, double2 *f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= o.N) return;
    const int p = o.p, n = o.n, G2 = o.G2, NL = o.nl;
    const int32_t *in = o.inc + (size_t)i * 2 * 5;
    const int j = in[0], i1 = in[2], i2 = in[3];
    double2 acc = make_double2(0, 0);
    for (int e2 = max(0, i2 - p); e2 <= min(n - 1, i2); ++e2)
        for (int e1 = max(0, i1 - p); e1 <= min(n - 1, i1); ++e1) {
            const int l = (i2 - e2) * (p + 1) + (i1 - e1);
            const int64_t e = ((int64_t)j * n + e2) * n + e1;
            const double *X = o.eX + e * 3 * G2;
            const double *Ps = o.ePsi + (e * 4 + 3) * NL * G2 + (size_t)l * G2;   // weight * value * |J|
            for (int q = 0; q < G2; ++q) {
                double2 g;
                if (kind == 0) {
                    double sn, cs;
                    sincos(o.kappa * (a0 * X[q] + a1 * X[G2 + q] + a2 * X[2 * G2 + q]), &sn, &cs);
                    g = make_double2(cs, sn);
                } else {
                    const double d0 = X[q] - a0, d1 = X[G2 + q] - a1, d2 = X[2 * G2 + q] - a2;
                    g = helmholtz(o.kappa, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
                }
                acc = cadd(acc, cscale(Ps[q], g));
            }
        }
    f[i] = acc;
}

__global__ void k_helmholtz_eval(int64_t n, double kappa, const double *r2, double2 *out, int prec,
                                 const double2 *sctab)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (prec == IGE_F32) out[i] = dm::to_d(dm::helmholtz_r2((float)kappa, (float)r2[i]));
    else out[i] = dm::helmholtz_r2_tab(kappa, r2[i], sctab);
}

}  // namespace

void launch_helmholtz_eval(hipStream_t s, int64_t n, double kappa, const double *r2, double2 *out, int prec,
                           const double2 *sctab)
{
    hipLaunchKernelGGL(k_helmholtz_eval, dim3((n + 255) / 256), dim3(256), 0, s, n, kappa, r2, out, prec, sctab);
    IGE_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define IGE_LAUNCH_CHECK() IGE_HIP(hipGetLastError())

void launch_element_data(ige_op op)
{
    const DevOp &o = op->view;
    const int64_t E = (int64_t)o.P * o.n * o.n;
    const int threads = 64;
    hipStream_t s = lstream(op);
#define IGE_ED(NLV) hipLaunchKernelGGL(k_element_data<NLV>, dim3(E), dim3(threads), 0, s, o, op->d_eX.p, op->d_ePsi.p, op->d_ePsiF.p, op->d_eC.p)
    switch (o.nl) {
        case 4: IGE_ED(4); break;
        case 9: IGE_ED(9); break;
        case 12: IGE_ED(12); break;
        case 16: IGE_ED(16); break;
        case 24: IGE_ED(24); break;
        case 25: IGE_ED(25); break;
        default: IGE_ED(40); break;
    }
#undef IGE_ED
    IGE_LAUNCH_CHECK();
}

void launch_node_geometry(ige_op op)
{
    const DevOp &o = op->view;
    const int64_t tot = (int64_t)op->NC * o.Q;
    hipLaunchKernelGGL(k_node_geometry, dim3((tot + 255) / 256), dim3(256), 0, lstream(op), o, op->NC,
                       op->d_nodeX.p, op->d_nodeT.p);
    IGE_LAUNCH_CHECK();
}

size_t psi_fragment_doubles(int nl, int G2)
{
    const int LT = (nl + 15) / 16, QT = (G2 + 15) / 16;
    return (size_t)4 * LT * 4 * QT * 64;
}

namespace {
template <int NL>
void launch_near_regular_nl(ige_op op, dim3 grid, size_t shm, int sb, int ce1, int ce2, int cs1, int cs2, int sstep)
{
    const DevOp &o = op->view;
    hipStream_t s = lstream(op);
    switch ((o.G2 + 15) / 16) {
        case 1:
            if constexpr (NL <= 12) hipLaunchKernelGGL((k_near_regular_o2<NL, 1>), grid, dim3(256), shm, s, o, sb, ce1, ce2, cs1, cs2, sstep);
            else hipLaunchKernelGGL((k_near_regular<NL, 1>), grid, dim3(256), shm, s, o, sb, ce1, ce2, cs1, cs2, sstep);
            break;
        case 2:
            if constexpr (NL <= 12) hipLaunchKernelGGL((k_near_regular_o2<NL, 2>), grid, dim3(256), shm, s, o, sb, ce1, ce2, cs1, cs2, sstep);
            else hipLaunchKernelGGL((k_near_regular<NL, 2>), grid, dim3(256), shm, s, o, sb, ce1, ce2, cs1, cs2, sstep);
            break;
        case 3: hipLaunchKernelGGL((k_near_regular<NL, 3>), grid, dim3(256), shm, s, o, sb, ce1, ce2, cs1, cs2, sstep); break;
        default: hipLaunchKernelGGL((k_near_regular<NL, 4>), grid, dim3(256), shm, s, o, sb, ce1, ce2, cs1, cs2, sstep); break;
    }
}
}  // namespace

// shared memory of k_near_regular: block rows of the test element over a trial
// square of sb x sb elements, and four staged element-pair blocks
size_t near_regular_shm(int sb, int p, int nl)
{
    const size_t nr = nl <= 24 ? nl : 16 * near_regular_lr(nl);   // rows per workgroup
    return sizeof(double2) * (nr * 2 * (sb + p) * (sb + p) + (size_t)4 * nr * nl);
}

int near_regular_sb(int s, int p, int nl)
{
    // trial squares of sb x sb elements: the largest power of two <= s that fits in
    // 64 KB of shared memory
    int sb = s;
    while (sb > 1 && near_regular_shm(sb, p, nl) > 64 * 1024) sb /= 2;
    return sb;
}

void launch_near_regular(ige_op op)
{
    const DevOp &o = op->view;
    if (o.nblk == 0) return;
    IGE_REQUIRE(o.G2 <= 64, "regular near-field rule limited to 8 x 8 points");
    const int sb = near_regular_sb(o.s, o.p, o.nl);
    const int nsb = o.s / sb;
    // colours: test elements p + 1 apart (a glued function spans at most p + 1
    // elements per direction); with several trial squares per leaf, squares whose gap
    // of (sstep - 1) sb elements is at least p
    const int P1 = o.p + 1, sstep = nsb > 1 ? 1 + (o.p + sb - 1) / sb : 1;
    const size_t shm = near_regular_shm(sb, o.p, o.nl);
    for (int ce2 = 0; ce2 < std::min(P1, o.s); ++ce2)
        for (int ce1 = 0; ce1 < std::min(P1, o.s); ++ce1)
            for (int cs2 = 0; cs2 < std::min(sstep, nsb); ++cs2)
                for (int cs1 = 0; cs1 < std::min(sstep, nsb); ++cs1) {
                    const int64_t n1 = (o.s - ce1 + P1 - 1) / P1, n2 = (o.s - ce2 + P1 - 1) / P1;
                    const int64_t m1 = (nsb - cs1 + sstep - 1) / sstep, m2 = (nsb - cs2 + sstep - 1) / sstep;
                    const int LT = (o.nl + 15) / 16;
                    const int64_t nrt = LT / near_regular_lr(o.nl);   // row-tile workgroups per element
                    const int64_t nwg = o.nblk * n1 * n2 * m1 * m2 * nrt;
                    if (nwg == 0) continue;
                    const dim3 grid((unsigned)nwg);
                    switch (o.nl) {
                        case 4: launch_near_regular_nl<4>(op, grid, shm, sb, ce1, ce2, cs1, cs2, sstep); break;
                        case 9: launch_near_regular_nl<9>(op, grid, shm, sb, ce1, ce2, cs1, cs2, sstep); break;
                        case 12: launch_near_regular_nl<12>(op, grid, shm, sb, ce1, ce2, cs1, cs2, sstep); break;
                        case 16: launch_near_regular_nl<16>(op, grid, shm, sb, ce1, ce2, cs1, cs2, sstep); break;
                        case 24: launch_near_regular_nl<24>(op, grid, shm, sb, ce1, ce2, cs1, cs2, sstep); break;
                        case 25: launch_near_regular_nl<25>(op, grid, shm, sb, ce1, ce2, cs1, cs2, sstep); break;
                        default: launch_near_regular_nl<40>(op, grid, shm, sb, ce1, ce2, cs1, cs2, sstep); break;
                    }
                    IGE_LAUNCH_CHECK();
                }
}

void launch_near_singular(ige_op op)
{
    const DevOp &o = op->view;
    if (op->nsing == 0) return;
    hipStream_t s = lstream(op);
    if (o.scalar) {
        switch (o.p) {
            case 1: hipLaunchKernelGGL((k_near_singular<1, true>), dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
            case 2: hipLaunchKernelGGL((k_near_singular<2, true>), dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
            case 3: hipLaunchKernelGGL((k_near_singular<3, true>), dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
            default: hipLaunchKernelGGL((k_near_singular<4, true>), dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
        }
    } else {
        switch (o.p) {
            case 1: hipLaunchKernelGGL(k_near_singular<1>, dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
            case 2: hipLaunchKernelGGL(k_near_singular<2>, dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
            case 3: hipLaunchKernelGGL(k_near_singular<3>, dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
            default: hipLaunchKernelGGL(k_near_singular<4>, dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
        }
    }
    IGE_LAUNCH_CHECK();
}

void launch_p2m(ige_op op, const double2 *x)
{
    const DevOp &o = op->view;
    const int nleaf = o.P * o.SL * o.SL;
    if (o.scalar) {
        const size_t W = o.s + o.p;
        const size_t shm = sizeof(double2) * (W * W + W * o.Q1);
        hipLaunchKernelGGL(k_p2m_sc, dim3(nleaf), dim3(256), shm, lstream(op), o, x, op->d_mom.p, op->d_src.p);
        IGE_LAUNCH_CHECK();
        return;
    }
    const int w1a = o.s + o.p, w2a = o.s + o.p - 1;
    const size_t shm = sizeof(double2) * (2 * w1a * w2a + 3 * (size_t)(w1a) * o.Q1);
    hipLaunchKernelGGL(k_p2m, dim3(nleaf), dim3(256), shm, lstream(op), o, x, op->d_mom.p, op->d_src.p);
    IGE_LAUNCH_CHECK();
}

void launch_m2m(ige_op op)
{
    const DevOp &o = op->view;
    const size_t shm = sizeof(double2) * 24 * o.Q;
    lds_attr_once(reinterpret_cast<const void *>(&k_m2m), shm);
    // parents down to the coarsest level with far pairs (coarser moments are unused)
    for (int lvl = o.L - 1; lvl >= std::max(0, op->lfar); --lvl) {
        const int ncl = o.P << (2 * lvl);
        hipLaunchKernelGGL(k_m2m, dim3(ncl), dim3(256), shm, lstream(op), o, lvl, op->d_mom.p, op->d_src.p);
        IGE_LAUNCH_CHECK();
    }
    if (!o.varq) return;
    // levels of a smaller degree: source fields from the restricted moments
    for (int lvl = std::max(0, op->lfar); lvl <= o.L; ++lvl) {
        const int Q1l = o.ql[lvl] + 1;
        if (Q1l == o.Q1) continue;
        const size_t sh = sizeof(double2) * (3 * (size_t)o.Q + 3 * (size_t)o.Q1 * Q1l);
        hipLaunchKernelGGL(k_restrict, dim3(o.P << (2 * lvl)), dim3(256), sh, lstream(op), o, lvl, op->d_mom.p,
                           op->d_src.p);
        IGE_LAUNCH_CHECK();
    }
}

// dynamic shared memory above the 64 KB granted without asking (degrees 12..15 of the
// transfer kernels): the kernel's limit is raised once, before any graph capture
void lds_attr_once(const void *kern, size_t shm)
{
    if (shm <= (size_t)64 * 1024) return;
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> lk(mu);
    size_t &have = done[kern];
    if (have >= shm) return;
    IGE_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    have = shm;
}

size_t m2l_sym_shared_bytes(int Q)
{
    const int TPG = (Q + kM2LNT - 1) / kM2LNT;
    const int S = std::min(kM2LThreads / TPG, Q);
    // [Q][4] positions, two [Q][4] complex, then a chunk of G or the reduction of two fields
    return sizeof(double) * 4 * Q + sizeof(double2) * 8 * Q + sizeof(double2) * std::max((size_t)Q * TPG, (size_t)2 * S * Q);
}

size_t m2l_shared_bytes(int Q)
{
    const int TPG = (Q + kM2LNT - 1) / kM2LNT;
    const int S = std::min(kM2LThreads / TPG, Q);
    // [Q][4] positions + [Q][4] complex, or the reduction of two fields
    return std::max(sizeof(double) * 4 * Q + sizeof(double2) * 4 * Q, sizeof(double2) * 2 * (size_t)Q * S);
}

void launch_m2l(ige_op op, int prec)
{
    const DevOp &o = op->view;
    if (op->work.empty()) return;
    if (op->stored && !op->m2l_generate_one) {
        m2l_stored_one(op, prec);
        return;
    }
    if (op->m2l_sym && prec == IGE_F64) {
        const size_t shm = m2l_sym_shared_bytes(o.Q);
        lds_attr_once(reinterpret_cast<const void *>(&k_m2l_sym), shm);
        const int nw = (int)op->swork.size();
        hipLaunchKernelGGL(k_m2l_sym, dim3(nw), dim3(kM2LThreads), shm, lstream(op), o, nw, op->d_swork.p,
                           op->d_spartner.p, op->d_src.p, op->d_spart.p);
        IGE_LAUNCH_CHECK();
        return;
    }
    size_t shm = m2l_shared_bytes(o.Q);   // the largest over the levels' node counts
    for (int lvl = 0; lvl <= o.L; ++lvl) shm = std::max(shm, m2l_shared_bytes((o.ql[lvl] + 1) * (o.ql[lvl] + 1)));
    shm = std::max(shm, op->m2l_lds);
    // k = IGE_M2L_PERSIST workgroups per CU loop over the work items (room for the near
    // field's workgroups beside them); 0 (default): one workgroup per item
    const int nwork = (int)op->work1.size();
    int grid = nwork;
    if (op->m2l_persist > 0) {
        int ncu = 0;
        IGE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, op->ctx->device));
        grid = std::max(1, std::min(nwork, ncu * op->m2l_persist));
    }
    if (prec == IGE_F32) {
        lds_attr_once(reinterpret_cast<const void *>(&k_m2l<float>), shm);
        hipLaunchKernelGGL(k_m2l<float>, dim3(grid), dim3(kM2LThreads), shm, lstream(op), o, nwork,
                           op->d_work1.p, op->d_partner.p, op->d_src.p, op->d_part.p);
    } else {
        lds_attr_once(reinterpret_cast<const void *>(&k_m2l<double>), shm);
        hipLaunchKernelGGL(k_m2l<double>, dim3(grid), dim3(kM2LThreads), shm, lstream(op), o, nwork,
                           op->d_work1.p, op->d_partner.p, op->d_src.p, op->d_part.p);
    }
    IGE_LAUNCH_CHECK();
}

void launch_m2l_reduce(ige_op op, int prec)
{
    const DevOp &o = op->view;
    if (op->stored && !op->m2l_generate_one) {
        m2l_stored_reduce_one(op);
        return;
    }
    if (op->m2l_sym && prec == IGE_F64) {
        const int nt = std::min(512, (4 * o.Q + 63) / 64 * 64);
        hipLaunchKernelGGL(k_m2l_reduce_sym, dim3(op->NC), dim3(nt), 0, lstream(op), o, op->d_sred_ptr.p,
                           op->d_sred_idx.p, op->d_spart.p, op->d_loc.p);
        IGE_LAUNCH_CHECK();
        return;
    }
    hipLaunchKernelGGL(k_m2l_reduce, dim3(op->NC), dim3(128), 0, lstream(op), o, op->d_wrk_of_tgt1.p,
                       op->d_part.p, op->d_loc.p);
    IGE_LAUNCH_CHECK();
    if (!o.varq) return;
    // levels of a smaller degree: local expansions back to the degree-q nodes
    for (int lvl = std::max(0, op->lfar); lvl <= o.L; ++lvl) {
        const int Q1l = o.ql[lvl] + 1;
        if (Q1l == o.Q1) continue;
        const size_t sh = sizeof(double2) * (3 * (size_t)Q1l * Q1l + 3 * (size_t)Q1l * o.Q1);
        hipLaunchKernelGGL(k_lift, dim3(o.P << (2 * lvl)), dim3(256), sh, lstream(op), o, lvl, op->d_loc.p);
        IGE_LAUNCH_CHECK();
    }
}

void launch_l2l(ige_op op)
{
    const DevOp &o = op->view;
    const size_t shm = sizeof(double2) * 3 * o.Q;
    // children below the coarsest level with far pairs (the expansions above it are zero)
    for (int lvl = std::max(1, op->lfar + 1); lvl <= o.L; ++lvl) {
        const int ncl = o.P << (2 * lvl);
        hipLaunchKernelGGL(k_l2l, dim3(ncl), dim3(256), shm, lstream(op), o, lvl, op->d_loc.p);
        IGE_LAUNCH_CHECK();
    }
}

int near_blk_u(int nF)
{
    const int u = (nF + 63) / 64;
    for (int c : {1, 2, 3, 4, 6, 8, 12, 16})
        if (u <= c) return c;
    return 16;
}

void launch_spmv(ige_op op, const double2 *x, double2 *y, hipStream_t st, hipEvent_t mid)
{
    const DevOp &o = op->view;
    if (o.nblk == 0) {
        IGE_HIP(hipMemsetAsync(y, 0, sizeof(double2) * o.N, st));
        if (mid) IGE_HIP(hipEventRecord(mid, st));
        return;
    }
    if (op->cmp_on) {
        double2 *part = op->d_cpart.p;
        launch_near_once(op, x, part, st);
        if (mid) IGE_HIP(hipEventRecord(mid, st));
        hipLaunchKernelGGL(k_near_gather, dim3((unsigned)(((int64_t)o.N * 16 + 255) / 256)), dim3(256), 0, st, o.N,
                           op->d_cred_ptr.p, op->d_cred_idx.p, part, y);
        IGE_LAUNCH_CHECK();
        return;
    }
    const dim3 grid((unsigned)(o.nblk * o.nch)), blk(256);
    double2 *part = op->d_npart.p;
    switch (near_blk_u(o.nF)) {
        case 1: hipLaunchKernelGGL(k_near_blk<1>, grid, blk, 0, st, o, x, part); break;
        case 2: hipLaunchKernelGGL(k_near_blk<2>, grid, blk, 0, st, o, x, part); break;
        case 3: hipLaunchKernelGGL(k_near_blk<3>, grid, blk, 0, st, o, x, part); break;
        case 4: hipLaunchKernelGGL(k_near_blk<4>, grid, blk, 0, st, o, x, part); break;
        case 6: hipLaunchKernelGGL(k_near_blk<6>, grid, blk, 0, st, o, x, part); break;
        case 8: hipLaunchKernelGGL(k_near_blk<8>, grid, blk, 0, st, o, x, part); break;
        case 12: hipLaunchKernelGGL(k_near_blk<12>, grid, blk, 0, st, o, x, part); break;
        default: hipLaunchKernelGGL(k_near_blk<16>, grid, blk, 0, st, o, x, part); break;
    }
    IGE_LAUNCH_CHECK();
    if (mid) IGE_HIP(hipEventRecord(mid, st));
    hipLaunchKernelGGL(k_near_gather, dim3((unsigned)(((int64_t)o.N * 16 + 255) / 256)), dim3(256), 0, st, o.N, o.red_ptr, o.red_idx, part, y);
    IGE_LAUNCH_CHECK();
}

void launch_l2p_leaf(ige_op op)
{
    const DevOp &o = op->view;
    const int nleaf = o.P * o.SL * o.SL;
    if (o.scalar) {
        const size_t shm = sizeof(double2) * (size_t)o.Q1 * (o.s + o.p);
        hipLaunchKernelGGL(k_l2p_leaf_sc, dim3(nleaf), dim3(256), shm, lstream(op), o, op->d_loc.p, op->d_ybuf.p);
        IGE_LAUNCH_CHECK();
        return;
    }
    const size_t shm = sizeof(double2) * 3 * (size_t)o.Q1 * o.rowlen;
    hipLaunchKernelGGL(k_l2p_leaf, dim3(nleaf), dim3(256), shm, lstream(op), o, op->d_loc.p, op->d_ybuf.p);
    IGE_LAUNCH_CHECK();
}

void launch_l2p_gather(ige_op op, double2 *y)
{
    const DevOp &o = op->view;
    hipLaunchKernelGGL(k_l2p_gather, dim3((o.N + 255) / 256), dim3(256), 0, lstream(op), o, op->d_ybuf.p, y);
    IGE_LAUNCH_CHECK();
}

void launch_rhs_scalar(ige_op op, int kind, const double *a, double2 *f)
{
    const DevOp &o = op->view;
    hipLaunchKernelGGL(k_rhs_scalar, dim3((o.N + 255) / 256), dim3(256), 0, lstream(op), o, kind, a[0], a[1], a[2], f);
    IGE_LAUNCH_CHECK();
}

void launch_rhs_plane(ige_op op, const double *dir, double2 pol0, double2 pol1, double2 pol2, double2 *f)
{
    const DevOp &o = op->view;
    hipLaunchKernelGGL(k_rhs_plane, dim3((o.N + 127) / 128), dim3(128), 0, lstream(op), o, dir[0], dir[1], dir[2],
                       pol0, pol1, pol2, f);
    IGE_LAUNCH_CHECK();
}

}  // namespace ige

// ---------------------------------------------------------------------------
// Scattered field e_s = V~ w at points off the surface (Sec. 2, eq. (eq:ESLP)):
//   e_s(x) = sum_e sum_q [G(x - y_q) W_q + kappa^-2 grad_x G(x - y_q) D_q],
// W_q = sum_l w_l Psi_l(q) (weighted phi_hat^a d_aF), D_q = sum_l w_l div_l(q), on the
// regular g x g Gauss points of every element; grad_x G = (x - y) G (i kappa r - 1) / r^2.
// ---------------------------------------------------------------------------
namespace ige {
namespace {

// per element Gauss point: y (3), W (3 complex), D (complex) -> src[E*G2][kPotStride]
constexpr int kPotStride = 11;

template <int NL>
__global__ void k_pot_sources(DevOp o, const double2 *w, double *src)
{
    const int64_t e = blockIdx.x;
    const int G2 = o.G2;
    int j, e1, e2;
    elem_of(o, e, j, e1, e2);
    double2 cf[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        int idx;
        double sg;
        local_dof(o, j, e1, e2, l, idx, sg);
        cf[l] = idx >= 0 ? cscale(sg, w[idx]) : make_double2(0.0, 0.0);
    }
    for (int q = threadIdx.x; q < G2; q += blockDim.x) {
        double *s = src + ((size_t)e * G2 + q) * kPotStride;
        for (int d = 0; d < 3; ++d) s[d] = o.eX[((size_t)e * 3 + d) * G2 + q];
        for (int c = 0; c < 4; ++c) {
            double2 W = make_double2(0.0, 0.0);
#pragma unroll
            for (int l = 0; l < NL; ++l) W = cadd(W, cscale(o.ePsi[(((size_t)e * 4 + c) * NL + l) * G2 + q], cf[l]));
            s[3 + 2 * c] = W.x;
            s[4 + 2 * c] = W.y;
        }
    }
}

// one workgroup per target point; threads take every 256th source point, then a
// fixed tree over the workgroup
// scalar: the single layer potential u(x) = int G(x - y) w(y) dsigma into component 0
__global__ __launch_bounds__(256) void k_potential(int64_t nsrc, double kappa, const double *src, const double *pts,
                                                   double2 *out, int scalar)
{
    __shared__ double red[6][256];
    const int t = blockIdx.x;
    const double x0 = pts[3 * t], x1 = pts[3 * t + 1], x2 = pts[3 * t + 2];
    const double ik2 = 1.0 / (kappa * kappa);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = threadIdx.x; i < nsrc; i += blockDim.x) {
        const double *s = src + i * kPotStride;
        const double rv[3] = {x0 - s[0], x1 - s[1], x2 - s[2]};
        const double rr2 = fma(rv[0], rv[0], fma(rv[1], rv[1], rv[2] * rv[2]));
        const double kr = kappa * sqrt(rr2);
        const double2 G = dm::helmholtz_r2(kappa, rr2);
        if (scalar) {
            const double2 v = cmul(G, make_double2(s[9], s[10]));
            acc[0] += v.x;
            acc[1] += v.y;
            continue;
        }
        // grad_x G = (x - y) G (i kappa r - 1) / r^2, times kappa^-2 and D
        const double2 dG = make_double2((-G.x - kr * G.y) / rr2, (kr * G.x - G.y) / rr2);
        const double2 dgD = cscale(ik2, cmul(dG, make_double2(s[9], s[10])));
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double2 v = cadd(cmul(G, make_double2(s[3 + 2 * d], s[4 + 2 * d])), cscale(rv[d], dgD));
            acc[2 * d] += v.x;
            acc[2 * d + 1] += v.y;
        }
    }
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[3 * t + threadIdx.x] = make_double2(red[2 * threadIdx.x][0], red[2 * threadIdx.x + 1][0]);
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of ige_potential_noalloc: the per-element source data of the
// potential (kPotStride doubles per Gauss point of every element), at most
// kPotScratchDoubles doubles (64 MiB).  Every device the library runs on holds its
// own copy until the process ends.  Host code never passes the symbol itself: its
// device address is looked up once per device (potential_scratch_init, with that
// device current) and kept per device ordinal.
// ---------------------------------------------------------------------------
constexpr size_t kPotScratchDoubles = (size_t)8 << 20;
static __device__ __align__(256) double scratch[kPotScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;   // device address of scratch per device ordinal
}  // namespace

void potential_scratch_init(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    IGE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = static_cast<double *>(ptr);
}

double *potential_scratch(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

size_t potential_scratch_doubles() { return kPotScratchDoubles; }

size_t potential_source_doubles(ige_op op) { return (size_t)op->view.P * op->view.n * op->view.n * op->view.G2 * kPotStride; }

void launch_potential(ige_op op, const double2 *w, int npts, const double *pts, double2 *out, double *src)
{
    const DevOp &o = op->view;
    const int64_t E = (int64_t)o.P * o.n * o.n;
    hipStream_t s = lstream(op);
    switch (o.nl) {
        case 4: hipLaunchKernelGGL(k_pot_sources<4>, dim3((unsigned)E), dim3(64), 0, s, o, w, src); break;
        case 9: hipLaunchKernelGGL(k_pot_sources<9>, dim3((unsigned)E), dim3(64), 0, s, o, w, src); break;
        case 12: hipLaunchKernelGGL(k_pot_sources<12>, dim3((unsigned)E), dim3(64), 0, s, o, w, src); break;
        case 16: hipLaunchKernelGGL(k_pot_sources<16>, dim3((unsigned)E), dim3(64), 0, s, o, w, src); break;
        case 24: hipLaunchKernelGGL(k_pot_sources<24>, dim3((unsigned)E), dim3(64), 0, s, o, w, src); break;
        case 25: hipLaunchKernelGGL(k_pot_sources<25>, dim3((unsigned)E), dim3(64), 0, s, o, w, src); break;
        default: hipLaunchKernelGGL(k_pot_sources<40>, dim3((unsigned)E), dim3(64), 0, s, o, w, src); break;
    }
    IGE_HIP(hipGetLastError());
    if (npts > 0) {
        hipLaunchKernelGGL(k_potential, dim3(npts), dim3(256), 0, s, E * o.G2, o.kappa, src, pts, out, o.scalar);
        IGE_HIP(hipGetLastError());
    }
}

}  // namespace ige
