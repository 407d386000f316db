// Stored coupling blocks of the far field (set-up and M2L).
//
// Every admissible cluster pair appears in both orders, and the interpolated
// kernel matrix of (s, t) is the transpose of that of (t, s): G_ts[m][m'] =
// G(|x_t,m - x_s,m'|).  One block is stored per unordered pair (t < s) and applied
// in both directions from a single read:
//   u_t[m]  += sum_m' G[m][m'] v_s[m']     (row side)
//   u_s[m'] += sum_m  G[m][m'] v_t[m]      (column side)
// for the four Cartesianised fields v = (v_x, v_y, v_z, d).  Every pair writes its
// two partial results; a per-cluster list sums them in a fixed order and converts
// to the test-side fields t^a = d_aF . u_xyz, t^d = -kappa^-2 u_d.
//
// Layouts: G [pair][m][m'] complex (FP64, optional FP32 copy); cluster fields
// [cluster][field][Q][r]; partials [2 pair + side][field][Q][RB] for the RB
// columns of one pass.
#include <hip/hip_runtime.h>

#include "device_math.hpp"
#include "op.hpp"

namespace ige {

namespace {

constexpr int kWave = 64;
typedef double d2v __attribute__((ext_vector_type(2)));

// kernel matrix entries of every stored pair
__global__ void k_g_store(DevOp o, int64_t nfp, const int32_t *fpair, double2 *G)
{
    const int Q = o.Q;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nfp * Q * Q) return;
    const int64_t pr = t / ((int64_t)Q * Q);
    const int r = (int)(t % ((int64_t)Q * Q)), m = r / Q, ms = r % Q;
    const double *Xt = o.nodeX + (size_t)fpair[2 * pr] * 3 * Q;
    const double *Xs = o.nodeX + (size_t)fpair[2 * pr + 1] * 3 * Q;
    const double d0 = Xt[m] - Xs[ms], d1 = Xt[Q + m] - Xs[Q + ms], d2 = Xt[2 * Q + m] - Xs[2 * Q + ms];
    G[t] = dm::helmholtz_r2_tab(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2)), o.sctab);
}

__global__ void k_g_to32(int64_t n, const double2 *G, float2 *G32)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) G32[t] = make_float2((float)G[t].x, (float)G[t].y);
}

__device__ inline d2v load_g(const double2 *p) { return __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p)); }
__device__ inline d2v load_g(const float2 *p)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
    return d2v{(double)v.x, (double)v.y};
}

// One workgroup per stored pair; wave w takes the rows m = w, w + 4, ...; lanes own
// the columns m' = lane + 64 u.  Row sums are reduced across the wave by halving;
// column sums accumulate in registers and are combined over the waves in order.
template <int U, int RB, typename TG>
__global__ __launch_bounds__(256) void k_m2l_g(DevOp o, int r, int c0, const int32_t *fpair, const TG *G,
                                               const double2 *src, double2 *part)
{
    constexpr int NV = 8 * RB;   // doubles per row result: 4 fields x RB columns x (re, im)
    __shared__ double2 svt[4][64 * U][RB];   // row-cluster fields, by row m
    __shared__ double2 scol[64 * U][4][RB];  // column partials, combined wave by wave
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int Q = o.Q;
    const int64_t pr = blockIdx.x;
    const int gt = fpair[2 * pr], gs = fpair[2 * pr + 1];
    const int nc = min(RB, r - c0);
    d2v vs[U][4][RB], ca[U][4][RB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int ms = lane + 64 * u;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                const double2 v = (ms < Q && j < nc) ? src[(((size_t)gs * 4 + f) * Q + ms) * r + c0 + j]
                                                     : make_double2(0.0, 0.0);
                vs[u][f][j] = d2v{v.x, v.y};
                ca[u][f][j] = d2v{0.0, 0.0};
            }
    }
    for (int i = threadIdx.x; i < 4 * Q * RB; i += blockDim.x) {
        const int j = i % RB, m = (i / RB) % Q, f = i / (RB * Q);
        svt[f][m][j] = j < nc ? src[(((size_t)gt * 4 + f) * Q + m) * r + c0 + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const TG *Gp = G + (size_t)pr * Q * Q;
    double *prow = reinterpret_cast<double *>(part + (size_t)(2 * pr) * 4 * Q * RB);
    // rows m and m + 4 per step: 2U streaming loads in flight per lane
    for (int m0 = wv; m0 < Q; m0 += 8) {
        d2v g[2][U];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int m = m0 + 4 * h, ms = lane + 64 * u;
                g[h][u] = (ms < Q && m < Q) ? load_g(Gp + (size_t)m * Q + ms) : d2v{0.0, 0.0};
            }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = m0 + 4 * h;
            if (m >= Q) break;   // uniform over the wave
            double a[NV];
#pragma unroll
            for (int f = 0; f < 4; ++f)
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    double re = 0.0, im = 0.0;
                    const double2 vt = svt[f][m][j];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const d2v gg = g[h][u];
                        re = fma(gg.x, vs[u][f][j].x, fma(-gg.y, vs[u][f][j].y, re));
                        im = fma(gg.x, vs[u][f][j].y, fma(gg.y, vs[u][f][j].x, im));
                        ca[u][f][j].x = fma(gg.x, vt.x, fma(-gg.y, vt.y, ca[u][f][j].x));
                        ca[u][f][j].y = fma(gg.x, vt.y, fma(gg.y, vt.x, ca[u][f][j].y));
                    }
                    a[2 * (f * RB + j)] = re;
                    a[2 * (f * RB + j) + 1] = im;
                }
            const double tot = dm::Halve<NV>::run(a, lane, 32);
            constexpr int SH = 6 - dm::log2c<NV>();
            if ((lane & ((1 << SH) - 1)) == 0) {
                const int k = lane >> SH, comp = k & 1, fj = k >> 1, f = fj / RB, j = fj % RB;
                prow[(((size_t)f * Q + m) * RB + j) * 2 + comp] = tot;
            }
        }
    }
    // column side: waves add their partials in the order 0, 1, 2, 3
    for (int w = 0; w < 4; ++w) {
        if (wv == w)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ms = lane + 64 * u;
                if (ms < Q)
#pragma unroll
                    for (int f = 0; f < 4; ++f)
#pragma unroll
                        for (int j = 0; j < RB; ++j) {
                            const double2 prev = w == 0 ? make_double2(0.0, 0.0) : scol[ms][f][j];
                            scol[ms][f][j] = make_double2(prev.x + ca[u][f][j].x, prev.y + ca[u][f][j].y);
                        }
            }
        __syncthreads();
    }
    double2 *pcol = part + (size_t)(2 * pr + 1) * 4 * Q * RB;
    for (int i = threadIdx.x; i < 4 * Q * RB; i += blockDim.x) {
        const int j = i % RB, ms = (i / RB) % Q, f = i / (RB * Q);
        pcol[i] = scol[ms][f][j];
    }
}

// Single column.  Wave w takes a quarter of the rows; a lane (h, c) = (lane / 32,
// lane % 32) takes the rows m = mb + 2 i + h and the columns m' = c + 32 k (k < KC), so
// a row of G is read by 32 lanes as one contiguous line and the source fields of the
// lane's columns stay in registers.  Row results are reduced over the 32 lanes of a
// half-wave (halving); column results accumulate in registers over all rows and
// are added over the two halves and then the four waves (fixed order).
constexpr int kQMax = 160;

template <int KC, typename TG>
__global__ __launch_bounds__(256) void k_m2l_t(DevOp o, const int32_t *fpair, const TG *G, const double2 *src,
                                               double2 *part)
{
    __shared__ double2 svt[4][kQMax];
    __shared__ double2 scol[4][kQMax];
    __shared__ double srow[4][kQMax][2];   // row results, written out after the loop
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, c = lane & 31;
    const int Q = o.Q;
    const int64_t pr = blockIdx.x;
    const int gt = fpair[2 * pr], gs = fpair[2 * pr + 1];
    d2v vs[KC][4], cp[KC][4];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int ms = c + 32 * k;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double2 v = ms < Q ? src[((size_t)gs * 4 + f) * Q + ms] : make_double2(0.0, 0.0);
            vs[k][f] = d2v{v.x, v.y};
            cp[k][f] = d2v{0.0, 0.0};
        }
    }
    for (int i = threadIdx.x; i < 4 * Q; i += blockDim.x) svt[i / Q][i % Q] = src[(size_t)gt * 4 * Q + i];
    __syncthreads();
    const TG *Gp = G + (size_t)pr * Q * Q;
    const int RW = (Q + 3) / 4, mb = wv * RW, me = min(Q, mb + RW);
    const int nit = (me - mb + 1) / 2;
    // rows are prefetched kDepth steps ahead into a rotating register buffer
    constexpr int kDepth = 4;
    d2v gb[kDepth][KC];
    auto load_row = [&](int it, d2v *dst) {
        const int m = mb + 2 * it + h;
        const bool ok = it < nit && m < me;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int ms = c + 32 * k;
            dst[k] = (ok && ms < Q) ? load_g(Gp + (size_t)m * Q + ms) : d2v{0.0, 0.0};
        }
    };
#pragma unroll
    for (int d = 0; d < kDepth; ++d) load_row(d, gb[d]);
    for (int it0 = 0; it0 < nit; it0 += kDepth) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d) {
            const int it = it0 + d;
            if (it >= nit) break;   // uniform over the wave
            const int m = mb + 2 * it + h;
            const bool ok = m < me;
            double a[8];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const double2 vt = ok ? svt[f][m] : make_double2(0.0, 0.0);
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const d2v g = gb[d][k];
                    re = fma(g.x, vs[k][f].x, fma(-g.y, vs[k][f].y, re));
                    im = fma(g.x, vs[k][f].y, fma(g.y, vs[k][f].x, im));
                    cp[k][f].x = fma(g.x, vt.x, fma(-g.y, vt.y, cp[k][f].x));
                    cp[k][f].y = fma(g.x, vt.y, fma(g.y, vt.x, cp[k][f].y));
                }
                a[2 * f] = re;
                a[2 * f + 1] = im;
            }
            load_row(it + kDepth, gb[d]);
            // halving over offsets 16, 8, 4, then full steps 2, 1: value (lane >> 2) & 7
            const double tot = dm::Halve<8>::run(a, lane, 16);
            if (ok && (lane & 3) == 0) {
                const int kk = (lane >> 2) & 7;
                srow[kk >> 1][m][kk & 1] = tot;
            }
        }
    }
    // column side: the two halves, then the waves in order 0..3
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            cp[k][f].x += __shfl_xor(cp[k][f].x, 32, kWave);
            cp[k][f].y += __shfl_xor(cp[k][f].y, 32, kWave);
        }
    for (int w = 0; w < 4; ++w) {
        if (wv == w && h == 0)
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const int ms = c + 32 * k;
                if (ms < Q)
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        const double2 prev = w == 0 ? make_double2(0.0, 0.0) : scol[f][ms];
                        scol[f][ms] = make_double2(prev.x + cp[k][f].x, prev.y + cp[k][f].y);
                    }
            }
        __syncthreads();
    }
    double2 *prow = part + (size_t)(2 * pr) * 4 * Q;
    double2 *pcol = prow + 4 * Q;
    for (int i = threadIdx.x; i < 4 * Q; i += blockDim.x) {
        prow[i] = make_double2(srow[i / Q][i % Q][0], srow[i / Q][i % Q][1]);
        pcol[i] = scol[i / Q][i % Q];
    }
}

// Per cluster, the sum of its partial couplings in list order, in two stages:
// stage 1 sums the kSplit interleaved sub-lists (entry k goes to sub-list k mod
// kSplit) per (cluster, sub-list) into tmp; stage 2 adds the sub-lists in order and
// converts to the test-side fields t^1, t^2, t^d for the RB columns of the pass.
constexpr int kSplit = 8;

template <int RB>
__global__ void k_m2l_sum_g(DevOp o, const int64_t *ptr, const int32_t *idx, const double2 *part, double2 *tmp)
{
    const int gc = blockIdx.x / kSplit, sl = blockIdx.x % kSplit, Q = o.Q;
    const int64_t b = ptr[gc], e = ptr[gc + 1];
    for (int t = threadIdx.x; t < 4 * Q * RB; t += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int64_t w = b + sl; w < e; w += kSplit) {
            const double2 v = part[(size_t)idx[w] * 4 * Q * RB + t];
            re += v.x;
            im += v.y;
        }
        tmp[((size_t)gc * kSplit + sl) * 4 * Q * RB + t] = make_double2(re, im);
    }
}

template <int RB>
__global__ void k_m2l_reduce_g(DevOp o, int r, int c0, const double2 *tmp, double2 *loc)
{
    const int gc = blockIdx.x, Q = o.Q;
    const double ik2 = 1.0 / (o.kappa * o.kappa);
    const int nc = min(RB, r - c0);
    for (int t = threadIdx.x; t < Q * RB; t += blockDim.x) {
        const int mm = t / RB, j = t % RB;
        if (j >= nc) continue;
        double2 u[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
        for (int sl = 0; sl < kSplit; ++sl) {
            const double2 *P = tmp + ((size_t)gc * kSplit + sl) * 4 * Q * RB;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double2 v = P[((size_t)k * Q + mm) * RB + j];
                u[k] = make_double2(u[k].x + v.x, u[k].y + v.y);
            }
        }
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        double2 t1 = make_double2(0, 0), t2 = make_double2(0, 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            t1 = make_double2(t1.x + T[k * Q + mm] * u[k].x, t1.y + T[k * Q + mm] * u[k].y);
            t2 = make_double2(t2.x + T[(3 + k) * Q + mm] * u[k].x, t2.y + T[(3 + k) * Q + mm] * u[k].y);
        }
        double2 *L = loc + (size_t)gc * 3 * Q * r;
        if (o.scalar) {   // scalar: |J(x_m)| u (the target's surface element)
            const double Fu[3] = {T[mm], T[Q + mm], T[2 * Q + mm]}, Fv[3] = {T[3 * Q + mm], T[4 * Q + mm], T[5 * Q + mm]};
            const double J = dm::surf_elem(Fu, Fv);
            L[((size_t)0 * Q + mm) * r + c0 + j] = make_double2(0, 0);
            L[((size_t)1 * Q + mm) * r + c0 + j] = make_double2(0, 0);
            L[((size_t)2 * Q + mm) * r + c0 + j] = make_double2(J * u[3].x, J * u[3].y);
            continue;
        }
        L[((size_t)0 * Q + mm) * r + c0 + j] = t1;
        L[((size_t)1 * Q + mm) * r + c0 + j] = t2;
        L[((size_t)2 * Q + mm) * r + c0 + j] = make_double2(-ik2 * u[3].x, -ik2 * u[3].y);
    }
}

template <int RB>
void m2l_reduce_pass(ige_op op, int r, int c0, double2 *loc, hipStream_t s)
{
    const DevOp &o = op->view;
    hipLaunchKernelGGL(k_m2l_sum_g<RB>, dim3((unsigned)(op->NC * kSplit)), dim3(256), 0, s, o, op->d_fred_ptr.p,
                       op->d_fred_idx.p, op->d_gpart.p, op->d_gtmp.p);
    IGE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_m2l_reduce_g<RB>, dim3(op->NC), dim3(128), 0, s, o, r, c0, op->d_gtmp.p, loc);
    IGE_HIP(hipGetLastError());
}

template <int U, int RB, typename TG>
void m2l_g_pass(ige_op op, int r, const TG *G, const double2 *src, double2 *loc, hipStream_t s)
{
    const DevOp &o = op->view;
    for (int c0 = 0; c0 < r; c0 += RB) {
        hipLaunchKernelGGL((k_m2l_g<U, RB, TG>), dim3((unsigned)op->nfp), dim3(256), 0, s, o, r, c0,
                           op->d_fpair.p, G, src, op->d_gpart.p);
        IGE_HIP(hipGetLastError());
        m2l_reduce_pass<RB>(op, r, c0, loc, s);
    }
}

template <typename TG>
void m2l_g_dispatch(ige_op op, int r, const TG *G, const double2 *src, double2 *loc, hipStream_t s)
{
    const int U = (op->view.Q + 63) / 64;
    if (U == 1) {
        if (r == 1) m2l_g_pass<1, 1>(op, r, G, src, loc, s);
        else m2l_g_pass<1, 4>(op, r, G, src, loc, s);
    } else if (U == 2) {
        if (r == 1) m2l_g_pass<2, 1>(op, r, G, src, loc, s);
        else m2l_g_pass<2, 2>(op, r, G, src, loc, s);
    } else {
        m2l_g_pass<3, 1>(op, r, G, src, loc, s);
    }
}

}  // namespace

int coupling_rb_max(int Q) { return Q <= 64 ? 4 : (Q <= 128 ? 2 : 1); }

void store_coupling(ige_op op)
{
    const DevOp &o = op->view;
    const int64_t n = op->nfp * o.Q * o.Q;
    if (n == 0) return;
    hipLaunchKernelGGL(k_g_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, lstream(op), o, op->nfp,
                       op->d_fpair.p, op->d_G.p);
    IGE_HIP(hipGetLastError());
}

void ensure_coupling32(ige_op op)
{
    const int64_t n = op->nfp * op->view.Q * op->view.Q;
    if (op->d_G32.p || n == 0) return;
    op->d_G32.alloc(n);
    hipLaunchKernelGGL(k_g_to32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, lstream(op), n, op->d_G.p,
                       op->d_G32.p);
    IGE_HIP(hipGetLastError());
}

namespace {
template <typename TG>
void m2l_t_launch(ige_op op, const TG *G)
{
    const DevOp &o = op->view;
    const dim3 grid((unsigned)op->nfp), blk(256);
    hipStream_t s = lstream(op);
    const double2 *src = op->d_src.p;
    double2 *part = op->d_gpart.p;
    switch ((o.Q + 31) / 32) {
        case 1: hipLaunchKernelGGL((k_m2l_t<1, TG>), grid, blk, 0, s, o, op->d_fpair.p, G, src, part); break;
        case 2: hipLaunchKernelGGL((k_m2l_t<2, TG>), grid, blk, 0, s, o, op->d_fpair.p, G, src, part); break;
        case 3: hipLaunchKernelGGL((k_m2l_t<3, TG>), grid, blk, 0, s, o, op->d_fpair.p, G, src, part); break;
        case 4: hipLaunchKernelGGL((k_m2l_t<4, TG>), grid, blk, 0, s, o, op->d_fpair.p, G, src, part); break;
        default: hipLaunchKernelGGL((k_m2l_t<5, TG>), grid, blk, 0, s, o, op->d_fpair.p, G, src, part); break;
    }
    IGE_HIP(hipGetLastError());
}
}  // namespace

void m2l_stored_one(ige_op op, int prec)
{
    if (op->nfp == 0) return;
    if (prec == IGE_F32) {
        ensure_coupling32(op);
        m2l_t_launch(op, op->d_G32.p);
    } else {
        m2l_t_launch(op, op->d_G.p);
    }
}

void m2l_stored_reduce_one(ige_op op) { m2l_reduce_pass<1>(op, 1, 0, op->d_loc.p, lstream(op)); }

int coupling_split() { return kSplit; }

void m2l_stored(ige_op op, int r, int prec, const double2 *src, double2 *loc, hipStream_t s)
{
    if (op->nfp == 0) return;
    if (prec == IGE_F32) {
        ensure_coupling32(op);
        m2l_g_dispatch(op, r, op->d_G32.p, src, loc, s);
    } else {
        m2l_g_dispatch(op, r, op->d_G.p, src, loc, s);
    }
}

}  // namespace ige
