// HIP kernels of the igaefie library (gfx950, wave64).
//
//   a0  element_data / node_geometry : geometry from the rational Bezier form at the
//       regular Gauss points of every element and at the Chebyshev nodes of every cluster
//   a1  near_regular / near_singular : element-pair Galerkin quadrature of the near field,
//       accumulated into the glued CSR matrix
//   a3  p2m   leaf moments, fused with the gather x_super = T x (1-D factors of T)
//   a4  m2m   upward transfer of the moments (nested cluster bases)
//   a5  m2l   coupling of admissible cluster pairs with the interpolated kernel
//   a6  l2l   downward transfer
//   a7  l2p   test-side moments, fused with the scatter T^T
//   a8  spmv  near-field product
//   a9  rhs   plane-wave right-hand side
//   a10 GMRES vector kernels
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.hpp"
#include "op.hpp"

namespace ige {

namespace {

constexpr int kWave = 64;
__device__ __constant__ double kInv4Pi = 0.07957747154594767;   // 1/(4 pi)

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

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

// local glued function l of an element: (component, t1, t2)
__device__ inline void local_index(int p, int l, int &a, int &t1, int &t2)
{
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
template <int NL>
__device__ inline void local_values(const DevOp &o, int e1, int e2, double x, double y, const double Fu[3],
                                    const double Fv[3], double Phi[NL][3], double Dv[NL])
{
    double Pu[kMaxP + 1], dPu[kMaxP + 1], Qu[kMaxP + 1], Pv[kMaxP + 1], dPv[kMaxP + 1], Qv[kMaxP + 1];
    spline_pieces(o, e1, x, Pu, dPu, Qu);
    spline_pieces(o, e2, y, Pv, dPv, Qv);
    const int p = o.p;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        int a, t1, t2;
        local_index(p, l, a, t1, t2);
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
    const int p = o.p;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        int a, t1, t2;
        local_index(p, l, a, t1, t2);
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
    local_index(o.p, l, a, t1, t2);
    const size_t off = (((size_t)j * 2 + a) * o.nb + (e2 + t2)) * o.nb + (e1 + t1);
    idx = o.dof[off];
    sg = (double)o.sgn[off];
}

// CSR accumulate A[i][j] += v
__device__ inline void csr_add(const DevOp &o, int i, int jcol, double2 v)
{
    int64_t lo = o.rowptr[i], hi = o.rowptr[i + 1] - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (o.col[mid] < jcol) lo = mid + 1;
        else hi = mid;
    }
    // the pattern contains every (i, j) of a near element pair
    if (o.col[lo] != jcol) {
        atomicAdd(o.err, 1);
        return;
    }
    double *dst = reinterpret_cast<double *>(o.val + lo);
    atomicAdd(dst, v.x);
    atomicAdd(dst + 1, v.y);
}

// ---------------------------------------------------------------------------
// a0: element data at the regular Gauss points
// ---------------------------------------------------------------------------
template <int NL>
__global__ void k_element_data(DevOp o, double *eX, double *ePsi, double *eC)
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
        for (int l = 0; l < NL; ++l) {
            for (int d = 0; d < 3; ++d) ePsi[(((size_t)e * 4 + d) * NL + l) * G2 + q] = w * Phi[l][d];
            ePsi[(((size_t)e * 4 + 3) * NL + l) * G2 + q] = w * Dv[l];
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
    const int m1 = mm % o.Q1, m2 = mm / o.Q1;
    const double H = 1.0 / S;
    double X[3], Fu[3], Fv[3];
    bezier_eval(o.geo, j, (k1 + o.xn[m1]) * H, (k2 + o.xn[m2]) * H, X, Fu, Fv);
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

// ---------------------------------------------------------------------------
// a1: regular element pairs (no shared corner), one wavefront per element pair.
//   B[l][l'] = sum_c S_c sum_q Psi_l^c(q) sum_q' K(q,q') Psi'_l'^c(q'),
//   S = (1, 1, 1, -kappa^-2), weights folded into Psi.
// ---------------------------------------------------------------------------
constexpr int kQB = 16;   // test points per LDS block of kernel values

template <int NL>
__global__ __launch_bounds__(64) void k_near_regular(DevOp o, const int32_t *near)
{
    extern __shared__ double smem[];
    const int s2 = o.s * o.s;
    const int64_t blk = blockIdx.x;
    const int64_t lp = blk / ((int64_t)s2 * s2);
    const int r = (int)(blk % ((int64_t)s2 * s2));
    const int ti = r / s2, tj = r % s2;
    const int lt = near[2 * lp], ls = near[2 * lp + 1];
    const int SL = o.SL;
    const int jt = lt / (SL * SL), jr = lt % (SL * SL);
    const int js = ls / (SL * SL), jsr = ls % (SL * SL);
    const int te1 = (jr % SL) * o.s + ti % o.s, te2 = (jr / SL) * o.s + ti / o.s;
    const int fe1 = (jsr % SL) * o.s + tj % o.s, fe2 = (jsr / SL) * o.s + tj / o.s;
    const int64_t e = ((int64_t)jt * o.n + te2) * o.n + te1;
    const int64_t f = ((int64_t)js * o.n + fe2) * o.n + fe1;
    if (share_corner(o, e, f)) return;   // handled by the singular kernel

    const int G2 = o.G2, lane = threadIdx.x;
    double *Xa = smem;                    // [3][G2]
    double *Xb = Xa + 3 * G2;             // [3][G2]
    double2 *K = reinterpret_cast<double2 *>(Xb + 3 * G2);   // [kQB][G2]
    double2 *part = K + kQB * G2;         // [4][NL][NL]
    for (int i = lane; i < 3 * G2; i += kWave) {
        Xa[i] = o.eX[e * 3 * G2 + i];
        Xb[i] = o.eX[f * 3 * G2 + i];
    }
    const double *Pa = o.ePsi + e * 4 * NL * G2;
    const double *Pb = o.ePsi + f * 4 * NL * G2;
    const double ik2 = 1.0 / (o.kappa * o.kappa);

    constexpr int NC = 4 * NL;
    constexpr int NPL = (NC + kWave - 1) / kWave;   // combos per lane
    double2 acc[NPL][NL];
#pragma unroll
    for (int c = 0; c < NPL; ++c)
#pragma unroll
        for (int l = 0; l < NL; ++l) acc[c][l] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int q0 = 0; q0 < G2; q0 += kQB) {
        const int nq = min(kQB, G2 - q0);
        for (int i = lane; i < nq * G2; i += kWave) {
            const int qa = q0 + i / G2, qb = i % G2;
            const double d0 = Xa[qa] - Xb[qb], d1 = Xa[G2 + qa] - Xb[G2 + qb], d2 = Xa[2 * G2 + qa] - Xb[2 * G2 + qb];
            K[i] = dm::helmholtz_r2(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2)));
        }
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < NPL; ++cc) {
            const int combo = lane + cc * kWave;
            if (combo < NC) {
                const int c = combo / NL, lb = combo % NL;
                const double *pb = Pb + ((size_t)c * NL + lb) * G2;
                for (int qq = 0; qq < nq; ++qq) {
                    double2 z = make_double2(0.0, 0.0);
                    const double2 *Kr = K + qq * G2;
                    for (int qb = 0; qb < G2; ++qb) {
                        const double w = pb[qb];
                        z.x += Kr[qb].x * w;
                        z.y += Kr[qb].y * w;
                    }
                    const double *pa = Pa + (size_t)c * NL * G2 + q0 + qq;
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        const double a = pa[(size_t)l * G2];
                        acc[cc][l].x += a * z.x;
                        acc[cc][l].y += a * z.y;
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cc = 0; cc < NPL; ++cc) {
        const int combo = lane + cc * kWave;
        if (combo < NC) {
            const int c = combo / NL, lb = combo % NL;
            const double sc = (c == 3) ? -ik2 : 1.0;
#pragma unroll
            for (int l = 0; l < NL; ++l) part[((size_t)c * NL + l) * NL + lb] = cscale(sc, acc[cc][l]);
        }
    }
    __syncthreads();
    int jtp, a1, a2, jsp, b1, b2;
    elem_of(o, e, jtp, a1, a2);
    elem_of(o, f, jsp, b1, b2);
    for (int i = lane; i < NL * NL; i += kWave) {
        const int l = i / NL, lb = i % NL;
        double2 v = make_double2(0.0, 0.0);
        for (int c = 0; c < 4; ++c) v = cadd(v, part[((size_t)c * NL + l) * NL + lb]);
        int ri, cj;
        double sr, sc;
        local_dof(o, jtp, a1, a2, l, ri, sr);
        local_dof(o, jsp, b1, b2, lb, cj, sc);
        csr_add(o, ri, cj, cscale(sr * sc, v));
    }
}

// ---------------------------------------------------------------------------
// a1: element pairs sharing a corner (relative-coordinate / Duffy sub-rules),
// one wavefront per pair; rows of the block are produced in chunks of RCH.
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

// Singular pairs: the points of the sub-rules are processed in batches of 64; in a
// batch every lane evaluates geometry, local basis and kernel at one point into
// LDS, then the lanes accumulate the block entries over the batch.
template <int NL>
__global__ __launch_bounds__(64) void k_near_singular(DevOp o, const SingularPair *list)
{
    __shared__ double sPa[kWave][NL][4];   // test side:  w*K-independent values Phi (3), div
    __shared__ double sPb[kWave][NL][4];   // trial side
    __shared__ double2 sK[kWave];          // weight * kernel
    const SingularPair sp = list[blockIdx.x];
    const int lane = threadIdx.x;
    int ja, a1, a2, jb, b1, b2;
    elem_of(o, sp.e, ja, a1, a2);
    elem_of(o, sp.f, jb, b1, b2);
    const int gs = o.gs, g4 = gs * gs * gs * gs;
    const int nsub = sp.kind == 1 ? 8 : (sp.kind == 2 ? 6 : 4);
    const int npts = nsub * g4;
    const double ik2 = 1.0 / (o.kappa * o.kappa), h4 = o.h * o.h * o.h * o.h;
    constexpr int NE = (NL * NL + kWave - 1) / kWave;   // block entries per lane
    double2 acc[NE];
#pragma unroll
    for (int t = 0; t < NE; ++t) acc[t] = make_double2(0.0, 0.0);
    for (int p0 = 0; p0 < npts; p0 += kWave) {
        const int pt = p0 + lane;
        __syncthreads();   // the previous batch has been consumed
        if (pt < npts) {
            double s1, s2, t1, t2, wt;
            singular_point(o, sp.kind, pt, s1, s2, t1, t2, wt);
            double xa, ya, xb, yb;
            if (sp.kind == 1) {
                xa = s1; ya = s2; xb = t1; yb = t2;
            } else {
                frame_map(sp.fa, s1, s2, xa, ya);
                frame_map(sp.fb, t1, t2, xb, yb);
            }
            double XA[3], XB[3], Fu[3], Fv[3];
            bezier_eval(o.geo, ja, (a1 + xa) * o.h, (a2 + ya) * o.h, XA, Fu, Fv);
            local_values_lds<NL>(o, a1, a2, xa, ya, Fu, Fv, -ik2, sPa[lane]);
            bezier_eval(o.geo, jb, (b1 + xb) * o.h, (b2 + yb) * o.h, XB, Fu, Fv);
            local_values_lds<NL>(o, b1, b2, xb, yb, Fu, Fv, 1.0, sPb[lane]);
            const double d0 = XA[0] - XB[0], d1 = XA[1] - XB[1], d2 = XA[2] - XB[2];
            sK[lane] = cscale(wt * h4, dm::helmholtz_r2(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2))));
        }
        __syncthreads();
        const int nb = min(kWave, npts - p0);
#pragma unroll
        for (int t = 0; t < NE; ++t) {
            const int ent = lane + t * kWave;
            if (ent < NL * NL) {
                const int l = ent / NL, lb = ent % NL;
                double2 a = acc[t];
                for (int q = 0; q < nb; ++q) {
                    const double gsum = sPa[q][l][0] * sPb[q][lb][0] + sPa[q][l][1] * sPb[q][lb][1] +
                                        sPa[q][l][2] * sPb[q][lb][2] + sPa[q][l][3] * sPb[q][lb][3];
                    a.x = fma(sK[q].x, gsum, a.x);
                    a.y = fma(sK[q].y, gsum, a.y);
                }
                acc[t] = a;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NE; ++t) {
        const int ent = lane + t * kWave;
        if (ent < NL * NL) {
            const int l = ent / NL, lb = ent % NL;
            int ri, cj;
            double sr, sc;
            local_dof(o, ja, a1, a2, l, ri, sr);
            local_dof(o, jb, b1, b2, lb, cj, sc);
            csr_add(o, ri, cj, cscale(sr * sc, acc[t]));
        }
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
        Sv[3 * Q + mm] = d;
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

template <typename T>
__global__ __launch_bounds__(kM2LThreads) void k_m2l(DevOp o, const M2LWork *work, const int32_t *partner,
                                                      const double2 *src, double2 *part)
{
    using C = typename dm::cplx_of<T>::type;
    extern __shared__ double smd[];
    const M2LWork wk = work[blockIdx.x];
    const int Q = o.Q;
    const int TPG = (Q + kM2LNT - 1) / kM2LNT;
    const int S = min(kM2LThreads / TPG, Q);
    const int SP = (Q + S - 1) / S;
    const int tid = threadIdx.x;
    const int mt = tid % TPG, sp = tid / TPG;
    const bool active = sp < S;
    T *sX = reinterpret_cast<T *>(smd);                        // [3][Q]
    C *sV = reinterpret_cast<C *>(smd + (3 * Q * (int)sizeof(T) + 15) / 16 * 2);   // [4][Q], 16-B aligned after sX
    double2 *red = reinterpret_cast<double2 *>(smd);           // [S][Q][4] after the partner loop
    const T kap = (T)o.kappa;
    T xt[kM2LNT][3];
    bool val[kM2LNT];
    C acc[kM2LNT][4];
    const double *Xt = o.nodeX + (size_t)wk.tgt * 3 * Q;
#pragma unroll
    for (int k = 0; k < kM2LNT; ++k) {
        const int mm = mt + k * TPG;
        val[k] = active && mm < Q;
        const int mc = val[k] ? mm : 0;
        xt[k][0] = (T)Xt[mc];
        xt[k][1] = (T)Xt[Q + mc];
        xt[k][2] = (T)Xt[2 * Q + mc];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[k][j] = C{0, 0};
    }
    const int mb = min(Q, sp * SP), me = min(Q, mb + SP);
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const int sc = partner[kp];
        __syncthreads();
        const double *Xs = o.nodeX + (size_t)sc * 3 * Q;
        const double2 *Vs = src + (size_t)sc * 4 * Q;
        for (int i = tid; i < 3 * Q; i += kM2LThreads) sX[i] = (T)Xs[i];
        for (int i = tid; i < 4 * Q; i += kM2LThreads) sV[i] = dm::to_c(Vs[i], T(0));
        __syncthreads();
        if (active) {
            for (int ms = mb; ms < me; ++ms) {
                const T x0 = sX[ms], x1 = sX[Q + ms], x2 = sX[2 * Q + ms];
                const C v0 = sV[ms], v1 = sV[Q + ms], v2 = sV[2 * Q + ms], v3 = sV[3 * Q + ms];
#pragma unroll
                for (int k = 0; k < kM2LNT; ++k) {
                    const T d0 = xt[k][0] - x0, d1 = xt[k][1] - x1, d2 = xt[k][2] - x2;
                    const C G = dm::helmholtz_r2(kap, d0 * d0 + d1 * d1 + d2 * d2);
                    acc[k][0] = dm::cadd(acc[k][0], dm::cmul(G, v0));
                    acc[k][1] = dm::cadd(acc[k][1], dm::cmul(G, v1));
                    acc[k][2] = dm::cadd(acc[k][2], dm::cmul(G, v2));
                    acc[k][3] = dm::cadd(acc[k][3], dm::cmul(G, v3));
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kM2LNT; ++k)
        if (val[k]) {
            const int mm = mt + k * TPG;
#pragma unroll
            for (int j = 0; j < 4; ++j) red[((size_t)sp * Q + mm) * 4 + j] = dm::to_d(acc[k][j]);
        }
    __syncthreads();
    for (int i = tid; i < 4 * Q; i += kM2LThreads) {
        const int j = i / Q, mm = i % Q;
        double2 v = make_double2(0, 0);
        for (int q2 = 0; q2 < S; ++q2) v = cadd(v, red[((size_t)q2 * Q + mm) * 4 + j]);
        part[(size_t)blockIdx.x * 4 * Q + i] = v;
    }
}

// sum the partial couplings of every cluster (fixed order) and convert to the
// test-side fields t^a = d_aF . u_xyz, t^d = -kappa^-2 u_d
__global__ void k_m2l_reduce(DevOp o, const int32_t *wrk_of_tgt, const double2 *part, double2 *loc)
{
    const int gc = blockIdx.x, Q = o.Q;
    const int b = wrk_of_tgt[gc], e = wrk_of_tgt[gc + 1];
    const double ik2 = 1.0 / (o.kappa * o.kappa);
    for (int mm = threadIdx.x; mm < Q; mm += blockDim.x) {
        double2 u[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
        for (int w = b; w < e; ++w)
            for (int k = 0; k < 4; ++k) u[k] = cadd(u[k], part[((size_t)w * 4 + k) * Q + mm]);
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        double2 t1 = make_double2(0, 0), t2 = make_double2(0, 0);
        for (int k = 0; k < 3; ++k) {
            t1 = cadd(t1, cscale(T[k * Q + mm], u[k]));
            t2 = cadd(t2, cscale(T[(3 + k) * Q + mm], u[k]));
        }
        double2 *L = loc + (size_t)gc * 3 * Q;
        L[mm] = t1;
        L[Q + mm] = t2;
        L[2 * Q + mm] = cscale(-ik2, u[3]);
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
// a8: near-field SpMV, one wavefront per row
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spmv(DevOp o, const double2 *x, double2 *y)
{
    const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (row >= o.N) return;
    const int64_t b = o.rowptr[row], e = o.rowptr[row + 1];
    double re = 0.0, im = 0.0;
    // four independent streaming loads in flight per lane; the matrix is read once
    // per apply, so its loads bypass the caches (x stays cached)
    int64_t k = b + lane;
    for (; k + 3 * kWave < e; k += 4 * kWave) {
        typedef double d2v __attribute__((ext_vector_type(2)));
        d2v a[4];
        int c[4];
        const d2v *vv = reinterpret_cast<const d2v *>(o.val);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = __builtin_nontemporal_load(vv + k + u * kWave);
            c[u] = __builtin_nontemporal_load(&o.col[k + u * kWave]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 v = x[c[u]];
            re = fma(a[u].x, v.x, re);
            re = fma(-a[u].y, v.y, re);
            im = fma(a[u].x, v.y, im);
            im = fma(a[u].y, v.x, im);
        }
    }
    for (; k < e; k += kWave) {
        const double2 a = o.val[k];
        const double2 v = x[o.col[k]];
        re = fma(a.x, v.x, re);
        re = fma(-a.y, v.y, re);
        im = fma(a.x, v.y, im);
        im = fma(a.y, v.x, im);
    }
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off, kWave);
        im += __shfl_xor(im, off, kWave);
    }
    if (lane == 0) y[row] = make_double2(re, im);
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
        const int du = (a == 0) ? p : p - 1, dv = (a == 0) ? p - 1 : p;
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

// ---------------------------------------------------------------------------
// a10: GMRES vector kernels (deterministic reductions)
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

__device__ inline double2 block_reduce2(double2 v, double2 *sh)
{
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        v.x += __shfl_xor(v.x, off, kWave);
        v.y += __shfl_xor(v.y, off, kWave);
    }
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double2 r = make_double2(0, 0);
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) r = cadd(r, sh[i]);
    return r;
}

// out[k] = sum_i conj(V_k[i]) w[i], one block per k
__global__ __launch_bounds__(kRedThreads) void k_dotc(int64_t n, const double2 *V, int64_t ldv, const double2 *w,
                                                       double2 *out)
{
    __shared__ double2 sh[kRedThreads / kWave];
    const double2 *v = V + (size_t)blockIdx.x * ldv;
    double2 acc = make_double2(0, 0);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = v[i], b = w[i];
        acc.x += a.x * b.x + a.y * b.y;
        acc.y += a.x * b.y - a.y * b.x;
    }
    const double2 r = block_reduce2(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// w[i] -= sum_k V_k[i] h[k]
__global__ void k_gemv_sub(int64_t n, const double2 *V, int64_t ldv, int k, const double2 *hc, double2 *w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = w[i];
    for (int c = 0; c < k; ++c) {
        const double2 v = V[(size_t)c * ldv + i], hh = hc[c];
        acc.x -= v.x * hh.x - v.y * hh.y;
        acc.y -= v.x * hh.y + v.y * hh.x;
    }
    w[i] = acc;
}

__global__ void k_axpby(int64_t n, double2 a, const double2 *x, double2 b, double2 *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = cadd(cmul(a, x[i]), cmul(b, y[i]));
}

__global__ void k_scale_copy(int64_t n, double2 a, const double2 *x, double2 *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = cmul(a, x[i]);
}

__global__ __launch_bounds__(kRedThreads) void k_norm2(int64_t n, const double2 *x, double *out)
{
    __shared__ double2 sh[kRedThreads / kWave];
    double2 acc = make_double2(0, 0);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = x[i];
        acc.x += a.x * a.x + a.y * a.y;
    }
    const double2 r = block_reduce2(acc, sh);
    if (threadIdx.x == 0) out[0] = sqrt(r.x);
}

__global__ void k_helmholtz_eval(int64_t n, double kappa, const double *r2, double2 *out, int prec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (prec == IGE_F32) out[i] = dm::to_d(dm::helmholtz_r2((float)kappa, (float)r2[i]));
    else out[i] = dm::helmholtz_r2(kappa, r2[i]);
}

// ---- batched GMRES vector kernels: V is [k][r][N] (basis index, column, entry),
// W and X are [r][N]; per-column coefficients h are [r][hs]
__global__ __launch_bounds__(kRedThreads) void k_dotc_b(int64_t n, int r, const double2 *V, const double2 *w,
                                                         double2 *out, int hs)
{
    __shared__ double2 sh[kRedThreads / kWave];
    const int kk = blockIdx.x, c = blockIdx.y;
    const double2 *v = V + ((size_t)kk * r + c) * n;
    const double2 *wc = w + (size_t)c * n;
    double2 acc = make_double2(0, 0);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = v[i], b = wc[i];
        acc.x += a.x * b.x + a.y * b.y;
        acc.y += a.x * b.y - a.y * b.x;
    }
    const double2 res = block_reduce2(acc, sh);
    if (threadIdx.x == 0) out[(size_t)c * hs + kk] = res;
}

// w_c -= sum_{kk < k} V[kk][c] h[c][kk]
__global__ void k_gemv_sub_b(int64_t n, int r, const double2 *V, int k, const double2 *hc, int hs, double2 *w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n) return;
    double2 acc = w[(size_t)c * n + i];
    for (int kk = 0; kk < k; ++kk) {
        const double2 v = V[((size_t)kk * r + c) * n + i], hh = hc[(size_t)c * hs + kk];
        acc.x -= v.x * hh.x - v.y * hh.y;
        acc.y -= v.x * hh.y + v.y * hh.x;
    }
    w[(size_t)c * n + i] = acc;
}

__global__ __launch_bounds__(kRedThreads) void k_norm2_b(int64_t n, const double2 *x, double *out)
{
    __shared__ double2 sh[kRedThreads / kWave];
    const double2 *xc = x + (size_t)blockIdx.x * n;
    double2 acc = make_double2(0, 0);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = xc[i];
        acc.x += a.x * a.x + a.y * a.y;
    }
    const double2 res = block_reduce2(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(res.x);
}

// y_c = s_c x_c (s per column, real)
__global__ void k_scale_cols(int64_t n, const double *s, const double2 *x, double2 *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n) return;
    const double sc = s[c];
    const double2 v = x[(size_t)c * n + i];
    y[(size_t)c * n + i] = make_double2(sc * v.x, sc * v.y);
}

}  // namespace

void launch_dotc_b(ige_op op, int r, const double2 *V, int k, const double2 *w, double2 *out, int hs)
{
    hipLaunchKernelGGL(k_dotc_b, dim3(k, r), dim3(kRedThreads), 0, op->ctx->stream, (int64_t)op->view.N, r, V, w, out,
                       hs);
    IGE_HIP(hipGetLastError());
}

void launch_gemv_sub_b(ige_op op, int r, const double2 *V, int k, const double2 *hc, int hs, double2 *w)
{
    const int64_t n = op->view.N;
    hipLaunchKernelGGL(k_gemv_sub_b, dim3((n + 255) / 256, r), dim3(256), 0, op->ctx->stream, n, r, V, k, hc, hs, w);
    IGE_HIP(hipGetLastError());
}

void launch_norm2_b(ige_op op, int r, const double2 *x, double *out)
{
    hipLaunchKernelGGL(k_norm2_b, dim3(r), dim3(kRedThreads), 0, op->ctx->stream, (int64_t)op->view.N, x, out);
    IGE_HIP(hipGetLastError());
}

void launch_scale_cols(ige_op op, int r, const double *s, const double2 *x, double2 *y)
{
    const int64_t n = op->view.N;
    hipLaunchKernelGGL(k_scale_cols, dim3((n + 255) / 256, r), dim3(256), 0, op->ctx->stream, n, s, x, y);
    IGE_HIP(hipGetLastError());
}

void launch_helmholtz_eval(hipStream_t s, int64_t n, double kappa, const double *r2, double2 *out, int prec)
{
    hipLaunchKernelGGL(k_helmholtz_eval, dim3((n + 255) / 256), dim3(256), 0, s, n, kappa, r2, out, prec);
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
    hipStream_t s = op->ctx->stream;
    switch (o.p) {
        case 1: hipLaunchKernelGGL(k_element_data<4>, dim3(E), dim3(threads), 0, s, o, op->d_eX.p, op->d_ePsi.p, op->d_eC.p); break;
        case 2: hipLaunchKernelGGL(k_element_data<12>, dim3(E), dim3(threads), 0, s, o, op->d_eX.p, op->d_ePsi.p, op->d_eC.p); break;
        default: hipLaunchKernelGGL(k_element_data<24>, dim3(E), dim3(threads), 0, s, o, op->d_eX.p, op->d_ePsi.p, op->d_eC.p); break;
    }
    IGE_LAUNCH_CHECK();
}

void launch_node_geometry(ige_op op)
{
    const DevOp &o = op->view;
    const int64_t tot = (int64_t)op->NC * o.Q;
    hipLaunchKernelGGL(k_node_geometry, dim3((tot + 255) / 256), dim3(256), 0, op->ctx->stream, o, op->NC,
                       op->d_nodeX.p, op->d_nodeT.p);
    IGE_LAUNCH_CHECK();
}

void launch_near_regular(ige_op op, int64_t n_near)
{
    const DevOp &o = op->view;
    const int64_t s4 = (int64_t)o.s * o.s * o.s * o.s;
    const int64_t nblk = n_near * s4;
    if (nblk == 0) return;
    const size_t shm_base = sizeof(double) * 6 * o.G2 + sizeof(double2) * kQB * o.G2;
    hipStream_t s = op->ctx->stream;
    switch (o.p) {
        case 1:
            hipLaunchKernelGGL(k_near_regular<4>, dim3(nblk), dim3(64), shm_base + sizeof(double2) * 4 * 16, s, o,
                               op->d_near.p);
            break;
        case 2:
            hipLaunchKernelGGL(k_near_regular<12>, dim3(nblk), dim3(64), shm_base + sizeof(double2) * 4 * 144, s, o,
                               op->d_near.p);
            break;
        default:
            hipLaunchKernelGGL(k_near_regular<24>, dim3(nblk), dim3(64), shm_base + sizeof(double2) * 4 * 576, s, o,
                               op->d_near.p);
            break;
    }
    IGE_LAUNCH_CHECK();
}

void launch_near_singular(ige_op op)
{
    const DevOp &o = op->view;
    if (op->nsing == 0) return;
    hipStream_t s = op->ctx->stream;
    switch (o.p) {
        case 1: hipLaunchKernelGGL(k_near_singular<4>, dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
        case 2: hipLaunchKernelGGL(k_near_singular<12>, dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
        default: hipLaunchKernelGGL(k_near_singular<24>, dim3(op->nsing), dim3(64), 0, s, o, op->d_sing.p); break;
    }
    IGE_LAUNCH_CHECK();
}

void launch_p2m(ige_op op, const double2 *x)
{
    const DevOp &o = op->view;
    const int nleaf = o.P * o.SL * o.SL;
    const int w1a = o.s + o.p, w2a = o.s + o.p - 1;
    const size_t shm = sizeof(double2) * (2 * w1a * w2a + 3 * (size_t)(w1a) * o.Q1);
    hipLaunchKernelGGL(k_p2m, dim3(nleaf), dim3(256), shm, op->ctx->stream, o, x, op->d_mom.p, op->d_src.p);
    IGE_LAUNCH_CHECK();
}

void launch_m2m(ige_op op)
{
    const DevOp &o = op->view;
    const size_t shm = sizeof(double2) * 24 * o.Q;
    for (int lvl = o.L - 1; lvl >= 0; --lvl) {
        const int ncl = o.P << (2 * lvl);
        hipLaunchKernelGGL(k_m2m, dim3(ncl), dim3(256), shm, op->ctx->stream, o, lvl, op->d_mom.p, op->d_src.p);
        IGE_LAUNCH_CHECK();
    }
}

size_t m2l_shared_bytes(int Q)
{
    const int TPG = (Q + kM2LNT - 1) / kM2LNT;
    const int S = std::min(kM2LThreads / TPG, Q);
    // [3][Q] positions (16-byte aligned end) + [4][Q] complex, or the reduction
    return std::max(sizeof(double) * (3 * Q + 1) + sizeof(double2) * 4 * Q, sizeof(double2) * 4 * (size_t)Q * S);
}

void launch_m2l(ige_op op, int prec)
{
    const DevOp &o = op->view;
    if (op->work.empty()) return;
    if (prec == IGE_F32)
        hipLaunchKernelGGL(k_m2l<float>, dim3(op->work.size()), dim3(kM2LThreads), m2l_shared_bytes(o.Q),
                           op->ctx->stream, o, op->d_work.p, op->d_partner.p, op->d_src.p, op->d_part.p);
    else
        hipLaunchKernelGGL(k_m2l<double>, dim3(op->work.size()), dim3(kM2LThreads), m2l_shared_bytes(o.Q),
                           op->ctx->stream, o, op->d_work.p, op->d_partner.p, op->d_src.p, op->d_part.p);
    IGE_LAUNCH_CHECK();
}

void launch_m2l_reduce(ige_op op)
{
    const DevOp &o = op->view;
    hipLaunchKernelGGL(k_m2l_reduce, dim3(op->NC), dim3(128), 0, op->ctx->stream, o, op->d_wrk_of_tgt.p,
                       op->d_part.p, op->d_loc.p);
    IGE_LAUNCH_CHECK();
}

void launch_l2l(ige_op op)
{
    const DevOp &o = op->view;
    const size_t shm = sizeof(double2) * 3 * o.Q;
    for (int lvl = 1; lvl <= o.L; ++lvl) {
        const int ncl = o.P << (2 * lvl);
        hipLaunchKernelGGL(k_l2l, dim3(ncl), dim3(256), shm, op->ctx->stream, o, lvl, op->d_loc.p);
        IGE_LAUNCH_CHECK();
    }
}

void launch_spmv(ige_op op, const double2 *x, double2 *y, hipStream_t st)
{
    const DevOp &o = op->view;
    const int rows_per_block = 256 / kWave;
    hipLaunchKernelGGL(k_spmv, dim3((o.N + rows_per_block - 1) / rows_per_block), dim3(256), 0, st, o, x, y);
    IGE_LAUNCH_CHECK();
}

void launch_l2p_leaf(ige_op op)
{
    const DevOp &o = op->view;
    const int nleaf = o.P * o.SL * o.SL;
    const size_t shm = sizeof(double2) * 3 * (size_t)o.Q1 * o.rowlen;
    hipLaunchKernelGGL(k_l2p_leaf, dim3(nleaf), dim3(256), shm, op->ctx->stream, o, op->d_loc.p, op->d_ybuf.p);
    IGE_LAUNCH_CHECK();
}

void launch_l2p_gather(ige_op op, double2 *y)
{
    const DevOp &o = op->view;
    hipLaunchKernelGGL(k_l2p_gather, dim3((o.N + 255) / 256), dim3(256), 0, op->ctx->stream, o, op->d_ybuf.p, y);
    IGE_LAUNCH_CHECK();
}

void launch_rhs_plane(ige_op op, const double *dir, double2 pol0, double2 pol1, double2 pol2, double2 *f)
{
    const DevOp &o = op->view;
    hipLaunchKernelGGL(k_rhs_plane, dim3((o.N + 127) / 128), dim3(128), 0, op->ctx->stream, o, dir[0], dir[1], dir[2],
                       pol0, pol1, pol2, f);
    IGE_LAUNCH_CHECK();
}

void launch_dotc(ige_op op, const double2 *V, int64_t ldv, int k, const double2 *w, double2 *out)
{
    hipLaunchKernelGGL(k_dotc, dim3(k), dim3(kRedThreads), 0, op->ctx->stream, (int64_t)op->view.N, V, ldv, w, out);
    IGE_LAUNCH_CHECK();
}

void launch_gemv_sub(ige_op op, const double2 *V, int64_t ldv, int k, const double2 *hcoef, double2 *w)
{
    const int64_t n = op->view.N;
    hipLaunchKernelGGL(k_gemv_sub, dim3((n + 255) / 256), dim3(256), 0, op->ctx->stream, n, V, ldv, k, hcoef, w);
    IGE_LAUNCH_CHECK();
}

void launch_axpby(ige_op op, int64_t n, double2 a, const double2 *x, double2 b, double2 *y)
{
    hipLaunchKernelGGL(k_axpby, dim3((n + 255) / 256), dim3(256), 0, op->ctx->stream, n, a, x, b, y);
    IGE_LAUNCH_CHECK();
}

void launch_scale_copy(ige_op op, int64_t n, double2 a, const double2 *x, double2 *y)
{
    hipLaunchKernelGGL(k_scale_copy, dim3((n + 255) / 256), dim3(256), 0, op->ctx->stream, n, a, x, y);
    IGE_LAUNCH_CHECK();
}

void launch_norm2(ige_op op, int64_t n, const double2 *x, double *out)
{
    hipLaunchKernelGGL(k_norm2, dim3(1), dim3(kRedThreads), 0, op->ctx->stream, n, x, out);
    IGE_LAUNCH_CHECK();
}

}  // namespace ige
