// Vector kernels of the batched restarted complex GMRES that solves the
// compressed EFIE system without preconditioner (Sec. 5).
//
// Layouts: the Krylov basis V is [k][r][n] (basis index, column, entry), vectors w
// and X are [r][n].  Every reduction runs in a fixed order (per-wave sums over a
// fixed shuffle tree, then partials summed in index order by a second kernel), so
// an orthogonalisation step gives the same bits on every run.
//
// The basis is stored in FP64, or in FP32 for the inner solves of iterative
// refinement (the Gram-Schmidt passes then read half the bytes; every sum, the
// vector being orthogonalised and the solution stay FP64).
//
// Orthogonalisation is classical Gram-Schmidt with a selective second pass
// (Daniel-Gragg-Kaufman-Stewart): after w' = w - V V^H w, the pass is repeated for
// a column only when |w'|^2 < |w|^2 / 2, which keeps the basis orthogonal to
// working precision while a step usually reads V twice (dots, update) instead of
// four times.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.hpp"
#include "op.hpp"

namespace ige {

namespace {

constexpr int kWave = 64;
constexpr int kGsT = 16;     // entries per lane of the dot kernel: a chunk is 64 kGsT entries
constexpr int kGsE = 4;      // entries per thread of the update kernel: a block covers 256 kGsE
constexpr int kFillBlocks = 2048;

__device__ inline double2 wave_sum(double2 v)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        v.x += __shfl_xor(v.x, off, kWave);
        v.y += __shfl_xor(v.y, off, kWave);
    }
    return v;
}

__device__ inline double2 ld2(const double2 *p) { return *p; }
__device__ inline double2 ld2(const float2 *p)
{
    const float2 v = *p;
    return make_double2(v.x, v.y);
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// part[(c (k+1) + kk) nchk + ch] = sum over chunk ch of conj(V[kk][c][i]) w_c[i] for
// the basis indices kk of this block's group (blockIdx.z); slot kk = k holds |w_c|^2
// over the chunk.  One wave per basis index, each wave holding the chunk of w.
template <typename VT>
__global__ __launch_bounds__(256) void k_gs_dot(int64_t n, int r, const VT *V, int k, int kgs, const double2 *w,
                                                const int *gate, double2 *part, int nchk)
{
    const int c = blockIdx.y, ch = blockIdx.x, wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (!gate[c]) return;
    const int64_t i0 = (int64_t)ch * kWave * kGsT + lane;
    const double2 *wc = w + (size_t)c * n;
    double2 wl[kGsT];
#pragma unroll
    for (int t = 0; t < kGsT; ++t) {
        const int64_t i = i0 + (int64_t)kWave * t;
        wl[t] = i < n ? wc[i] : make_double2(0.0, 0.0);
    }
    const size_t slot0 = (size_t)c * (k + 1);
    const int k0 = blockIdx.z * kgs, k1 = min(k, k0 + kgs);
    // whole chunks load without bounds checks (all kGsT loads of a lane in flight)
    const bool full = (int64_t)(ch + 1) * kWave * kGsT <= n;
    for (int kk = k0 + wv; kk < k1; kk += 4) {
        const VT *v = V + ((size_t)kk * r + c) * n + i0;
        double2 vv[kGsT];
        if (full) {
#pragma unroll
            for (int t = 0; t < kGsT; ++t) vv[t] = ld2(v + kWave * t);
        } else {
#pragma unroll
            for (int t = 0; t < kGsT; ++t) vv[t] = i0 + kWave * t < n ? ld2(v + kWave * t) : make_double2(0.0, 0.0);
        }
        double2 a = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < kGsT; ++t) {
            a.x = fma(vv[t].x, wl[t].x, fma(vv[t].y, wl[t].y, a.x));
            a.y = fma(vv[t].x, wl[t].y, fma(-vv[t].y, wl[t].x, a.y));
        }
        a = wave_sum(a);
        if (lane == 0) part[(slot0 + kk) * nchk + ch] = a;
    }
    if (blockIdx.z == 0 && wv == 3) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < kGsT; ++t) s = fma(wl[t].x, wl[t].x, fma(wl[t].y, wl[t].y, s));
        s = wave_sum(s);
        if (lane == 0) part[(slot0 + k) * nchk + ch] = make_double2(s, 0.0);
    }
}

// h[c][kk] = sum_ch part[c][kk][ch] (kk < k) and nb[c] = sum_ch part[c][k][ch].x,
// one wave per (c, kk); columns with gate 0 get h = 0
__global__ __launch_bounds__(256) void k_gs_sum(int r, int k, int nchk, const double2 *part, const int *gate,
                                                double2 *h, int hs, double *nb)
{
    const int64_t id = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (id >= (int64_t)r * (k + 1)) return;
    const int c = (int)(id / (k + 1)), kk = (int)(id % (k + 1));
    double2 a = make_double2(0.0, 0.0);
    if (gate[c]) {
        const double2 *p = part + ((size_t)c * (k + 1) + kk) * nchk;
        for (int ch = lane; ch < nchk; ch += kWave) {
            a.x += p[ch].x;
            a.y += p[ch].y;
        }
        a = wave_sum(a);
    }
    if (lane != 0) return;
    if (kk < k) h[(size_t)c * hs + kk] = a;
    else if (nb && gate[c]) nb[c] = a.x;
}

// y_c -= sum_{kk in group} V[kk][c] h[c][kk] (sign -1) or += (sign +1).  With one
// group (gridDim.z == 1) the result goes to y in place and the block's |y_c|^2 to
// npart[c][block] (if npart); with several, group z writes its sum to
// split[z][c][i] for k_gs_comb.
template <typename VT>
__global__ __launch_bounds__(256) void k_gs_upd(int64_t n, int r, const VT *V, int k, int kgs, const double2 *h,
                                                int hs, double sign, const int *gate, double2 *y, double2 *split,
                                                double *npart, int nblk)
{
    __shared__ double sh[4];
    const int c = blockIdx.y;
    if (!gate[c]) return;
    const int64_t i0 = (int64_t)blockIdx.x * 256 * kGsE + threadIdx.x;
    const int k0 = blockIdx.z * kgs, k1 = min(k, k0 + kgs);
    double2 acc[kGsE];
#pragma unroll
    for (int e = 0; e < kGsE; ++e) acc[e] = make_double2(0.0, 0.0);
    const double2 *hc = h + (size_t)c * hs;
    // whole blocks: four basis vectors at a time with every load in flight
    const bool full = (int64_t)(blockIdx.x + 1) * 256 * kGsE <= n;
    int kk = k0;
    if (full)
        for (; kk + 4 <= k1; kk += 4) {
            double2 vv[4][kGsE], hh[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                hh[u] = hc[kk + u];
                const VT *v = V + ((size_t)(kk + u) * r + c) * n + i0;
#pragma unroll
                for (int e = 0; e < kGsE; ++e) vv[u][e] = ld2(v + 256 * e);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int e = 0; e < kGsE; ++e) {
                    acc[e].x = fma(vv[u][e].x, hh[u].x, fma(-vv[u][e].y, hh[u].y, acc[e].x));
                    acc[e].y = fma(vv[u][e].x, hh[u].y, fma(vv[u][e].y, hh[u].x, acc[e].y));
                }
        }
    for (; kk < k1; ++kk) {
        const double2 hh = hc[kk];
        const VT *v = V + ((size_t)kk * r + c) * n;
#pragma unroll
        for (int e = 0; e < kGsE; ++e) {
            const int64_t i = i0 + 256 * e;
            if (i < n) {
                const double2 vv = ld2(v + i);
                acc[e].x = fma(vv.x, hh.x, fma(-vv.y, hh.y, acc[e].x));
                acc[e].y = fma(vv.x, hh.y, fma(vv.y, hh.x, acc[e].y));
            }
        }
    }
    if (gridDim.z > 1) {
#pragma unroll
        for (int e = 0; e < kGsE; ++e) {
            const int64_t i = i0 + 256 * e;
            if (i < n) split[((size_t)blockIdx.z * r + c) * n + i] = acc[e];
        }
        return;
    }
    double s = 0.0;
    double2 *yc = y + (size_t)c * n;
#pragma unroll
    for (int e = 0; e < kGsE; ++e) {
        const int64_t i = i0 + 256 * e;
        if (i < n) {
            double2 t = yc[i];
            t.x = fma(sign, acc[e].x, t.x);
            t.y = fma(sign, acc[e].y, t.y);
            yc[i] = t;
            s = fma(t.x, t.x, fma(t.y, t.y, s));
        }
    }
    if (!npart) return;
    s = wave_sum(s);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) npart[(size_t)c * nblk + blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// y_c += sign sum_z split[z][c] (z in order), and the block's |y_c|^2 to npart
__global__ __launch_bounds__(256) void k_gs_comb(int64_t n, int r, int ng, const double2 *split, double sign,
                                                 const int *gate, double2 *y, double *npart, int nblk)
{
    __shared__ double sh[4];
    const int c = blockIdx.y;
    if (!gate[c]) return;
    const int64_t i0 = (int64_t)blockIdx.x * 256 * kGsE + threadIdx.x;
    double s = 0.0;
    double2 *yc = y + (size_t)c * n;
#pragma unroll
    for (int e = 0; e < kGsE; ++e) {
        const int64_t i = i0 + 256 * e;
        if (i >= n) continue;
        double2 a = make_double2(0.0, 0.0);
        for (int z = 0; z < ng; ++z) {
            const double2 v = split[((size_t)z * r + c) * n + i];
            a.x += v.x;
            a.y += v.y;
        }
        double2 t = yc[i];
        t.x = fma(sign, a.x, t.x);
        t.y = fma(sign, a.y, t.y);
        yc[i] = t;
        s = fma(t.x, t.x, fma(t.y, t.y, s));
    }
    if (!npart) return;
    s = wave_sum(s);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) npart[(size_t)c * nblk + blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// per column (one wave each): nf[c] = sum_b npart[c][b] for gate columns; then
// scal[c] = 1/sqrt(nf[c]) for run columns (0 otherwise) and, if flag, flag[c] =
// run[c] and nf[c] < nb[c] / 2 (the second-pass test)
__global__ __launch_bounds__(256) void k_gs_norm(int r, int nblk, const double *npart, const int *gate,
                                                 const int *run, const double *nb, double *nf, double *scal, int *flag)
{
    const int c = blockIdx.x * 4 + threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (c >= r) return;
    if (gate[c]) {
        double a = 0.0;
        for (int b = lane; b < nblk; b += kWave) a += npart[(size_t)c * nblk + b];
        a = wave_sum(a);
        if (lane == 0) nf[c] = a;
    }
    if (lane != 0) return;
    const double v = nf[c];
    if (gate[c] || !run[c]) scal[c] = (run[c] && v > 0.0) ? 1.0 / sqrt(v) : 0.0;
    if (flag) flag[c] = run[c] && v < 0.5 * nb[c];
}

// out[c][0..k) = h1[c] + h2[c], out[c][k] = (sqrt(nf[c]), 0): the new Hessenberg column
__global__ void k_gs_pack(int r, int k, const double2 *h1, const double2 *h2, int hs, const double *nf, double2 *out)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)r * (k + 1)) return;
    const int c = (int)(id / (k + 1)), kk = (int)(id % (k + 1));
    double2 v;
    if (kk < k) {
        const double2 a = h1[(size_t)c * hs + kk], b = h2[(size_t)c * hs + kk];
        v = make_double2(a.x + b.x, a.y + b.y);
    } else {
        v = make_double2(sqrt(nf[c]), 0.0);
    }
    out[id] = v;
}

// y = a x + b y; with b = 0 the old y is not read (it may hold anything, NaN included)
__global__ void k_axpby(int64_t n, double2 a, const double2 *x, double2 b, double2 *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 ax = dm::cmul(a, x[i]);
    y[i] = (b.x == 0.0 && b.y == 0.0) ? ax : dm::cadd(ax, dm::cmul(b, y[i]));
}

// out[c] = |x_c|, one block per column, fixed-order reduction
__global__ __launch_bounds__(256) void k_norm2_b(int64_t n, const double2 *x, double *out)
{
    __shared__ double sh[4];
    const double2 *xc = x + (size_t)blockIdx.x * n;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = xc[i];
        acc = fma(a.x, a.x, fma(a.y, a.y, acc));
    }
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(((sh[0] + sh[1]) + sh[2]) + sh[3]);
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

// y_c = s_c x_c and its FP32 copy v_c (s per column, real)
__global__ void k_scale_cols32(int64_t n, const double *s, const double2 *x, double2 *y, float2 *v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n) return;
    const double sc = s[c];
    const double2 a = x[(size_t)c * n + i];
    const double2 b = make_double2(sc * a.x, sc * a.y);
    y[(size_t)c * n + i] = b;
    v[(size_t)c * n + i] = make_float2((float)b.x, (float)b.y);
}

// y_c += s_c x_c (s per column, real)
__global__ void k_axpy_cols(int64_t n, const double *s, const double2 *x, double2 *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n) return;
    const double sc = s[c];
    if (sc == 0.0) return;
    const double2 v = x[(size_t)c * n + i];
    double2 &t = y[(size_t)c * n + i];
    t = make_double2(fma(sc, v.x, t.x), fma(sc, v.y, t.y));
}

int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace

GsPlan gs_plan(int64_t n, int r, int kmax)
{
    GsPlan g;
    g.nchk = cdiv(n, kWave * kGsT);
    g.nblk = cdiv(n, 256 * kGsE);
    // groups of basis indices so that a pass launches enough blocks to fill the chip
    g.dot_groups = std::max(1, std::min(cdiv(kFillBlocks, (int64_t)g.nchk * r), cdiv(kmax, 4)));
    g.upd_groups = std::max(1, std::min(cdiv(kFillBlocks, (int64_t)g.nblk * r), cdiv(kmax, 8)));
    return g;
}

size_t gs_part_count(const GsPlan &g, int r, int kmax) { return (size_t)r * (kmax + 1) * g.nchk; }
size_t gs_split_count(const GsPlan &g, int64_t n, int r) { return g.upd_groups > 1 ? (size_t)g.upd_groups * r * n : 0; }

namespace {
template <typename VT>
void gs_dots(hipStream_t s, const GsPlan &g, int64_t n, int r, const VT *V, int k, const double2 *w, const int *gate,
             double2 *part, double2 *h, int hs, double *nb)
{
    const int ng = std::max(1, std::min(g.dot_groups, cdiv(k, 4)));
    const int kgs = cdiv(k, ng);
    hipLaunchKernelGGL(k_gs_dot<VT>, dim3(g.nchk, r, ng), dim3(256), 0, s, n, r, V, k, kgs, w, gate, part, g.nchk);
    IGE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gs_sum, dim3(cdiv((int64_t)r * (k + 1), 4)), dim3(256), 0, s, r, k, g.nchk, part, gate, h, hs,
                       nb);
    IGE_HIP(hipGetLastError());
}

template <typename VT>
void gs_update(hipStream_t s, const GsPlan &g, int64_t n, int r, const VT *V, int k, const double2 *h, int hs,
               double sign, const int *gate, double2 *y, double2 *split, double *npart)
{
    const int ng = split ? std::max(1, std::min(g.upd_groups, cdiv(k, 8))) : 1;
    const int kgs = cdiv(k, ng);
    hipLaunchKernelGGL(k_gs_upd<VT>, dim3(g.nblk, r, ng), dim3(256), 0, s, n, r, V, k, kgs, h, hs, sign, gate, y,
                       split, npart, g.nblk);
    IGE_HIP(hipGetLastError());
    if (ng > 1) {
        hipLaunchKernelGGL(k_gs_comb, dim3(g.nblk, r), dim3(256), 0, s, n, r, ng, split, sign, gate, y, npart, g.nblk);
        IGE_HIP(hipGetLastError());
    }
}
}  // namespace

void launch_gs_dots(hipStream_t s, const GsPlan &g, int64_t n, int r, const double2 *V, int k, const double2 *w,
                    const int *gate, double2 *part, double2 *h, int hs, double *nb)
{
    gs_dots(s, g, n, r, V, k, w, gate, part, h, hs, nb);
}

void launch_gs_dots(hipStream_t s, const GsPlan &g, int64_t n, int r, const float2 *V, int k, const double2 *w,
                    const int *gate, double2 *part, double2 *h, int hs, double *nb)
{
    gs_dots(s, g, n, r, V, k, w, gate, part, h, hs, nb);
}

void launch_gs_update(hipStream_t s, const GsPlan &g, int64_t n, int r, const double2 *V, int k, const double2 *h,
                      int hs, double sign, const int *gate, double2 *y, double2 *split, double *npart)
{
    gs_update(s, g, n, r, V, k, h, hs, sign, gate, y, split, npart);
}

void launch_gs_update(hipStream_t s, const GsPlan &g, int64_t n, int r, const float2 *V, int k, const double2 *h,
                      int hs, double sign, const int *gate, double2 *y, double2 *split, double *npart)
{
    gs_update(s, g, n, r, V, k, h, hs, sign, gate, y, split, npart);
}

void launch_gs_norm(hipStream_t s, const GsPlan &g, int r, const double *npart, const int *gate, const int *run,
                    const double *nb, double *nf, double *scal, int *flag)
{
    hipLaunchKernelGGL(k_gs_norm, dim3(cdiv(r, 4)), dim3(256), 0, s, r, g.nblk, npart, gate, run, nb, nf, scal, flag);
    IGE_HIP(hipGetLastError());
}

void launch_gs_pack(hipStream_t s, int r, int k, const double2 *h1, const double2 *h2, int hs, const double *nf,
                    double2 *out)
{
    const int64_t tot = (int64_t)r * (k + 1);
    hipLaunchKernelGGL(k_gs_pack, dim3(cdiv(tot, 256)), dim3(256), 0, s, r, k, h1, h2, hs, nf, out);
    IGE_HIP(hipGetLastError());
}

void launch_axpby(ige_op op, int64_t n, double2 a, const double2 *x, double2 b, double2 *y)
{
    hipLaunchKernelGGL(k_axpby, dim3(cdiv(n, 256)), dim3(256), 0, op->ctx->stream, n, a, x, b, y);
    IGE_HIP(hipGetLastError());
}

void launch_norm2_b(ige_op op, int r, const double2 *x, double *out)
{
    hipLaunchKernelGGL(k_norm2_b, dim3(r), dim3(256), 0, op->ctx->stream, (int64_t)op->view.N, x, out);
    IGE_HIP(hipGetLastError());
}

void launch_axpy_cols(ige_op op, int r, const double *s, const double2 *x, double2 *y)
{
    const int64_t n = op->view.N;
    hipLaunchKernelGGL(k_axpy_cols, dim3(cdiv(n, 256), r), dim3(256), 0, op->ctx->stream, n, s, x, y);
    IGE_HIP(hipGetLastError());
}

void launch_scale_cols32(ige_op op, int r, const double *s, const double2 *x, double2 *y, float2 *v)
{
    const int64_t n = op->view.N;
    hipLaunchKernelGGL(k_scale_cols32, dim3(cdiv(n, 256), r), dim3(256), 0, op->ctx->stream, n, s, x, y, v);
    IGE_HIP(hipGetLastError());
}

void launch_scale_cols(ige_op op, int r, const double *s, const double2 *x, double2 *y)
{
    const int64_t n = op->view.N;
    hipLaunchKernelGGL(k_scale_cols, dim3(cdiv(n, 256), r), dim3(256), 0, op->ctx->stream, n, s, x, y);
    IGE_HIP(hipGetLastError());
}

}  // namespace ige
