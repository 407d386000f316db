// Batched (several right-hand sides) variants of the apply kernels.
//
// Layout: the r columns are innermost everywhere, x_t / y_t are [N][r], cluster
// arrays [cluster][field][Q][r]; a block handles a chunk of kRB columns
// (blockIdx.y), so the kernel values G of the coupling stage and the near-field
// block entries are read or computed once per chunk instead of once per column.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "device_math.hpp"
#include "op.hpp"

namespace ige {

namespace {

constexpr int kWave = 64;
constexpr int kRBMax = 8;   // largest column chunk

__device__ inline double2 cmulb(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 caddb(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cscaleb(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

__global__ void k_zero2(int64_t n, double2 *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = make_double2(0.0, 0.0);
}

// x [r][N] -> xt [N][r] and back
__global__ void k_to_rows(int64_t N, int r, const double2 *x, double2 *xt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * r) return;
    const int64_t i = t / r;
    const int c = (int)(t % r);
    xt[t] = x[(size_t)c * N + i];
}

__global__ void k_to_cols(int64_t N, int r, const double2 *yt, double2 *y)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * r) return;
    const int c = (int)(t / N);
    const int64_t i = t % N;
    y[t] = yt[i * r + c];
}

// the same through a 32 x 32 tile in LDS, so that both the loads and the stores run
// along contiguous memory (the direct kernels above stride one side by N or r);
// blocks of 256 threads over (N / 32, r / 32) tiles; TO_ROWS: x [r][N] -> xt [N][r]
constexpr int kTT = 32;
template <bool TO_ROWS>
__global__ __launch_bounds__(256) void k_transpose_t(int64_t N, int r, const double2 *in, double2 *out)
{
    __shared__ double2 tile[kTT][kTT + 1];
    const int64_t i0 = (int64_t)blockIdx.x * kTT;
    const int c0 = blockIdx.y * kTT, tx = threadIdx.x % kTT, ty = threadIdx.x / kTT;
    for (int k = ty; k < kTT; k += 256 / kTT) {
        if (TO_ROWS) {   // column c0 + k of x, entries i0 + tx
            const int c = c0 + k;
            const int64_t i = i0 + tx;
            if (c < r && i < N) tile[k][tx] = in[(size_t)c * N + i];
        } else {         // entry i0 + k of yt, columns c0 + tx
            const int c = c0 + tx;
            const int64_t i = i0 + k;
            if (c < r && i < N) tile[tx][k] = in[(size_t)i * r + c];
        }
    }
    __syncthreads();
    for (int k = ty; k < kTT; k += 256 / kTT) {
        if (TO_ROWS) {   // entry i0 + k of xt, columns c0 + tx
            const int c = c0 + tx;
            const int64_t i = i0 + k;
            if (c < r && i < N) out[(size_t)i * r + c] = tile[tx][k];
        } else {         // column c0 + k of y, entries i0 + tx
            const int c = c0 + k;
            const int64_t i = i0 + tx;
            if (c < r && i < N) out[(size_t)c * N + i] = tile[k][tx];
        }
    }
}

// ---------------------------------------------------------------------------
// near-field product over the stored blocks, RB columns per pass: every block
// entry is loaded once per pass and used for the RB columns of both the block and
// its transpose (same partial-result layout as one column, times RB)
// ---------------------------------------------------------------------------
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ inline double wave_sum_b(double v)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int U, int RB>
__global__ __launch_bounds__(256) void k_near_blk_b(DevOp o, int r, int c0, const double2 *xt, double2 *part)
{
    __shared__ double2 sxr[64 * U][RB];
    __shared__ double2 syc[64 * U][RB];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.x / o.nch;
    const int ch = blockIdx.x % o.nch;
    const int lt = o.bpair[2 * b], ls = o.bpair[2 * b + 1];
    const int nF = o.nF, r0 = ch * o.rc, r1 = min(nF, r0 + o.rc);
    const int nc = min(RB, r - c0);
    d2v xc[U][RB], yc[U][RB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int c = lane + 64 * u;
        const int d = c < nF ? o.leafdof[(size_t)ls * nF + c] : -1;
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const double2 v = (d >= 0 && j < nc) ? xt[(size_t)d * r + c0 + j] : make_double2(0.0, 0.0);
            xc[u][j] = d2v{v.x, v.y};
            yc[u][j] = d2v{0.0, 0.0};
        }
    }
    for (int k = threadIdx.x; k < (r1 - r0) * RB; k += blockDim.x) {
        const int row = k / RB, j = k % RB;
        const int d = o.leafdof[(size_t)lt * nF + r0 + row];
        sxr[row][j] = (d >= 0 && j < nc) ? xt[(size_t)d * r + c0 + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const d2v *B = reinterpret_cast<const d2v *>(o.bval) + (size_t)b * nF * nF;
    for (int rr = r0 + wv; rr < r1; rr += 4) {
        d2v a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = lane + 64 * u;
            a[u] = c < nF ? __builtin_nontemporal_load(B + (size_t)rr * nF + c) : d2v{0.0, 0.0};
        }
        double re[RB], im[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            re[j] = 0.0;
            im[j] = 0.0;
            const double2 xr = sxr[rr - r0][j];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                re[j] = fma(a[u].x, xc[u][j].x, fma(-a[u].y, xc[u][j].y, re[j]));
                im[j] = fma(a[u].x, xc[u][j].y, fma(a[u].y, xc[u][j].x, im[j]));
                yc[u][j].x = fma(a[u].x, xr.x, fma(-a[u].y, xr.y, yc[u][j].x));
                yc[u][j].y = fma(a[u].x, xr.y, fma(a[u].y, xr.x, yc[u][j].y));
            }
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            re[j] = wave_sum_b(re[j]);
            im[j] = wave_sum_b(im[j]);
        }
        if (lane == 0)
#pragma unroll
            for (int j = 0; j < RB; ++j) part[((size_t)b * nF + rr) * RB + j] = make_double2(re[j], im[j]);
    }
    if (lt == ls) return;   // diagonal block (uniform branch)
    // combine the waves' column partials in a fixed order
    for (int w = 0; w < 4; ++w) {
        if (wv == w)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lane + 64 * u;
                if (c < nF)
#pragma unroll
                    for (int j = 0; j < RB; ++j) {
                        const double2 prev = w == 0 ? make_double2(0.0, 0.0) : syc[c][j];
                        syc[c][j] = make_double2(prev.x + yc[u][j].x, prev.y + yc[u][j].y);
                    }
            }
        __syncthreads();
    }
    double2 *cp = part + ((size_t)o.nblk * nF + ((size_t)b * o.nch + ch) * nF) * RB;
    for (int k = threadIdx.x; k < nF * RB; k += blockDim.x) cp[k] = syc[k / RB][k % RB];
}

// 16 lanes per unknown (RB columns innermost), fixed butterfly over the 16
template <int RB>
__global__ __launch_bounds__(256) void k_near_gather_b(int N, int r, int c0, const int64_t *ptr,
                                                       const int32_t *idx, const double2 *part, double2 *yt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = (int)(t % RB), sub = (int)((t / RB) & 15);
    const int64_t i = t / (16 * RB);
    double re = 0.0, im = 0.0;
    if (i < N)
        for (int64_t k = ptr[i] + sub; k < ptr[i + 1]; k += 16) {
            const double2 v = part[(size_t)idx[k] * RB + j];
            re += v.x;
            im += v.y;
        }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off * RB, 16 * RB);
        im += __shfl_xor(im, off * RB, 16 * RB);
    }
    if (i < N && sub == 0 && c0 + j < r) yt[(size_t)i * r + c0 + j] = make_double2(re, im);
}

template <int U, int RB>
void near_batched_u(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s)
{
    const DevOp &o = op->view;
    for (int c0 = 0; c0 < r; c0 += RB) {
        hipLaunchKernelGGL((k_near_blk_b<U, RB>), dim3((unsigned)(o.nblk * o.nch)), dim3(256), 0, s, o, r, c0, xt,
                           op->d_bnpart.p);
        IGE_HIP(hipGetLastError());
        const int64_t tot = (int64_t)o.N * RB * 16;
        hipLaunchKernelGGL(k_near_gather_b<RB>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, o.N, r, c0,
                           o.red_ptr, o.red_idx, op->d_bnpart.p, yt);
        IGE_HIP(hipGetLastError());
    }
}

void near_batched(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s)
{
    const DevOp &o = op->view;
    if (o.nblk == 0) {
        const int64_t tot = (int64_t)o.N * r;
        hipLaunchKernelGGL(k_zero2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tot, yt);
        IGE_HIP(hipGetLastError());
        return;
    }
    switch (near_blk_u(o.nF)) {
        case 1: near_batched_u<1, 4>(op, r, xt, yt, s); break;
        case 2: near_batched_u<2, 4>(op, r, xt, yt, s); break;
        case 3: near_batched_u<3, 4>(op, r, xt, yt, s); break;
        case 4: near_batched_u<4, 4>(op, r, xt, yt, s); break;
        case 6: near_batched_u<6, 2>(op, r, xt, yt, s); break;
        case 8: near_batched_u<8, 2>(op, r, xt, yt, s); break;
        case 12: near_batched_u<12, 1>(op, r, xt, yt, s); break;
        default: near_batched_u<16, 1>(op, r, xt, yt, s); break;
    }
}

// ---------------------------------------------------------------------------
// P2M on the leaves (gather of the glued coefficients fused), kRB columns
// ---------------------------------------------------------------------------
template <int kRB>
__global__ __launch_bounds__(256) void k_p2m_b(DevOp o, int r, const double2 *xt, double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen;
    const int j = id / (SL * SL), rr = id % (SL * SL), k2 = rr / SL, k1 = rr % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    const int w1a = s + p, w2a = s + p - 1, w1b = s + p - 1, w2b = s + p;
    double2 *X1 = sm2;                         // [w2a][w1a][kRB]
    double2 *X2 = X1 + w2a * w1a * kRB;        // [w2b][w1b][kRB]
    double2 *Z1 = X2 + w2b * w1b * kRB;        // [w2a][Q1][kRB]
    double2 *Zd = Z1 + w2a * Q1 * kRB;
    double2 *Z2 = Zd + w2a * Q1 * kRB;         // [w2b][Q1][kRB]
    for (int i = threadIdx.x; i < w2a * w1a * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, i2 = t / w1a, i1 = t % w1a;
        const size_t off = (((size_t)j * 2 + 0) * o.nb + (k2 * s + i2)) * o.nb + (k1 * s + i1);
        X1[i] = c < nc ? cscaleb((double)o.sgn[off], xt[(size_t)o.dof[off] * r + c0 + c]) : make_double2(0, 0);
    }
    for (int i = threadIdx.x; i < w2b * w1b * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, i2 = t / w1b, i1 = t % w1b;
        const size_t off = (((size_t)j * 2 + 1) * o.nb + (k2 * s + i2)) * o.nb + (k1 * s + i1);
        X2[i] = c < nc ? cscaleb((double)o.sgn[off], xt[(size_t)o.dof[off] * r + c0 + c]) : make_double2(0, 0);
    }
    __syncthreads();
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mqu = o.Mq + (size_t)k1 * Q1 * RL, *Mdu = o.Mdp + (size_t)k1 * Q1 * RL;
    const double *Mpv = o.Mp + (size_t)k2 * Q1 * RL, *Mqv = o.Mq + (size_t)k2 * Q1 * RL, *Mdv = o.Mdp + (size_t)k2 * Q1 * RL;
    for (int i = threadIdx.x; i < w2a * Q1 * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, i2 = t / Q1, m1 = t % Q1;
        double2 z = make_double2(0, 0), zd = make_double2(0, 0);
        for (int i1 = 0; i1 < w1a; ++i1) {
            const double2 v = X1[(i2 * w1a + i1) * kRB + c];
            z = caddb(z, cscaleb(Mpu[m1 * RL + i1], v));
            zd = caddb(zd, cscaleb(Mdu[m1 * RL + i1], v));
        }
        Z1[i] = z;
        Zd[i] = zd;
    }
    for (int i = threadIdx.x; i < w2b * Q1 * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, i2 = t / Q1, m1 = t % Q1;
        double2 z = make_double2(0, 0);
        for (int i1 = 0; i1 < w1b; ++i1) z = caddb(z, cscaleb(Mqu[m1 * RL + i1], X2[(i2 * w1b + i1) * kRB + c]));
        Z2[i] = z;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Q * kRB; i += blockDim.x) {
        const int c = i % kRB, mm = i / kRB, m2 = mm / Q1, m1 = mm % Q1;
        if (c >= nc) continue;
        double2 s1 = make_double2(0, 0), s2v = make_double2(0, 0), d = make_double2(0, 0);
        for (int i2 = 0; i2 < w2a; ++i2) {
            s1 = caddb(s1, cscaleb(Mqv[m2 * RL + i2], Z1[(i2 * Q1 + m1) * kRB + c]));
            d = caddb(d, cscaleb(Mqv[m2 * RL + i2], Zd[(i2 * Q1 + m1) * kRB + c]));
        }
        for (int i2 = 0; i2 < w2b; ++i2) {
            s2v = caddb(s2v, cscaleb(Mpv[m2 * RL + i2], Z2[(i2 * Q1 + m1) * kRB + c]));
            d = caddb(d, cscaleb(Mdv[m2 * RL + i2], Z2[(i2 * Q1 + m1) * kRB + c]));
        }
        const size_t col = c0 + c;
        double2 *M = mom + (size_t)gc * 3 * Q * r;
        M[((size_t)0 * Q + mm) * r + col] = s1;
        M[((size_t)1 * Q + mm) * r + col] = s2v;
        M[((size_t)2 * Q + mm) * r + col] = d;
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        double2 *S = src + (size_t)gc * 4 * Q * r;
        for (int k = 0; k < 3; ++k)
            S[((size_t)k * Q + mm) * r + col] = caddb(cscaleb(T[k * Q + mm], s1), cscaleb(T[(3 + k) * Q + mm], s2v));
        S[((size_t)3 * Q + mm) * r + col] = d;
    }
}

// scalar single layer, kRB columns: leaf moments d = (M_p (x) M_p) c of the tensor
// B-spline coefficients over the leaf's W x W window (fields 0 and 1 zero) and the
// source values |J(x_m)| d at the nodes
template <int kRB>
__global__ __launch_bounds__(256) void k_p2m_sc_b(DevOp o, int r, const double2 *xt, double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen, W = s + p;
    const int j = id / (SL * SL), rr = id % (SL * SL), k2 = rr / SL, k1 = rr % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    double2 *X = sm2;                  // [W (i2)][W (i1)][kRB]
    double2 *Z = X + W * W * kRB;      // [W (i2)][Q1 (m1)][kRB]
    for (int i = threadIdx.x; i < W * W * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, i2 = t / W, i1 = t % W;
        const size_t off = ((size_t)j * 2 * o.nb + (k2 * s + i2)) * o.nb + (k1 * s + i1);
        X[i] = c < nc ? xt[(size_t)o.dof[off] * r + c0 + c] : make_double2(0, 0);
    }
    __syncthreads();
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mpv = o.Mp + (size_t)k2 * Q1 * RL;
    for (int i = threadIdx.x; i < W * Q1 * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, i2 = t / Q1, m1 = t % Q1;
        double2 z = make_double2(0, 0);
        for (int i1 = 0; i1 < W; ++i1) z = caddb(z, cscaleb(Mpu[m1 * RL + i1], X[(i2 * W + i1) * kRB + c]));
        Z[i] = z;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Q * kRB; i += blockDim.x) {
        const int c = i % kRB, mm = i / kRB, m2 = mm / Q1, m1 = mm % Q1;
        if (c >= nc) continue;
        double2 d = make_double2(0, 0);
        for (int i2 = 0; i2 < W; ++i2) d = caddb(d, cscaleb(Mpv[m2 * RL + i2], Z[(i2 * Q1 + m1) * kRB + c]));
        const size_t col = c0 + c;
        double2 *M = mom + (size_t)gc * 3 * Q * r;
        M[((size_t)0 * Q + mm) * r + col] = make_double2(0, 0);
        M[((size_t)1 * Q + mm) * r + col] = make_double2(0, 0);
        M[((size_t)2 * Q + mm) * r + col] = d;
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        const double Fu[3] = {T[mm], T[Q + mm], T[2 * Q + mm]}, Fv[3] = {T[3 * Q + mm], T[4 * Q + mm], T[5 * Q + mm]};
        double2 *S = src + (size_t)gc * 4 * Q * r;
        for (int k = 0; k < 3; ++k) S[((size_t)k * Q + mm) * r + col] = make_double2(0, 0);
        S[((size_t)3 * Q + mm) * r + col] = cscaleb(dm::surf_elem(Fu, Fv), d);
    }
}

// ---------------------------------------------------------------------------
// M2M, kRB columns
// ---------------------------------------------------------------------------
template <int kRB>
__global__ __launch_bounds__(256) void k_m2m_b(DevOp o, int lvl, int r, double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int S = 1 << lvl, Q1 = o.Q1, Q = o.Q;
    const int j = id / (S * S), rr = id % (S * S), k2 = rr / S, k1 = rr % S;
    const int gc = (int)o.lvl_off[lvl] + id;
    const int QR = Q * kRB;
    double2 *acc = sm2;               // [3 fields][Q][kRB]
    double2 *W = acc + 3 * QR;        // [3 fields][Q1 (n2)][Q1 (m1)][kRB] of one child
    double2 *X = W + 3 * QR;          // the child's three fields, staged at once (coalesced along columns)
    for (int i = threadIdx.x; i < 3 * QR; i += blockDim.x) acc[i] = make_double2(0, 0);
    for (int ch = 0; ch < 4; ++ch) {
        const int c1 = ch & 1, c2 = ch >> 1;
        const int cgc = (int)o.lvl_off[lvl + 1] + (j * 2 * S + 2 * k2 + c2) * 2 * S + 2 * k1 + c1;
        const double2 *cm = mom + (size_t)cgc * 3 * Q * r;
        const double *Tu = c1 ? o.T1 : o.T0, *Tv = c2 ? o.T1 : o.T0;
        __syncthreads();
        for (int i = threadIdx.x; i < 3 * QR; i += blockDim.x) {
            const int c = i % kRB, t = i / kRB;   // t = f Q + q
            X[i] = c < nc ? cm[(size_t)t * r + c0 + c] : make_double2(0, 0);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 3 * QR; i += blockDim.x) {
            const int c = i % kRB, t = i / kRB, f = t / Q, nm = t % Q, n2 = nm / Q1, m1 = nm % Q1;
            double2 z = make_double2(0, 0);
            for (int n1 = 0; n1 < Q1; ++n1)
                z = caddb(z, cscaleb(Tu[n1 * Q1 + m1], X[(f * Q + n2 * Q1 + n1) * kRB + c]));
            W[i] = z;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 3 * QR; i += blockDim.x) {
            const int c = i % kRB, t = i / kRB, f = t / Q, mm = t % Q, m2 = mm / Q1, m1 = mm % Q1;
            double2 z = acc[i];
            for (int n2 = 0; n2 < Q1; ++n2)
                z = caddb(z, cscaleb(Tv[n2 * Q1 + m2], W[(f * Q + n2 * Q1 + m1) * kRB + c]));
            acc[i] = z;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Q * kRB; i += blockDim.x) {
        const int c = i % kRB, mm = i / kRB;
        if (c >= nc) continue;
        const size_t col = c0 + c;
        const double2 s1 = acc[(0 * Q + mm) * kRB + c], s2v = acc[(1 * Q + mm) * kRB + c], d = acc[(2 * Q + mm) * kRB + c];
        double2 *M = mom + (size_t)gc * 3 * Q * r;
        M[((size_t)0 * Q + mm) * r + col] = s1;
        M[((size_t)1 * Q + mm) * r + col] = s2v;
        M[((size_t)2 * Q + mm) * r + col] = d;
        const double *T = o.nodeT + (size_t)gc * 6 * Q;
        double2 *Sv = src + (size_t)gc * 4 * Q * r;
        for (int k = 0; k < 3; ++k)
            Sv[((size_t)k * Q + mm) * r + col] = caddb(cscaleb(T[k * Q + mm], s1), cscaleb(T[(3 + k) * Q + mm], s2v));
        if (o.scalar) {   // scalar: the moments times the surface element at the node
            const double Fu[3] = {T[mm], T[Q + mm], T[2 * Q + mm]}, Fv[3] = {T[3 * Q + mm], T[4 * Q + mm], T[5 * Q + mm]};
            Sv[((size_t)3 * Q + mm) * r + col] = cscaleb(dm::surf_elem(Fu, Fv), d);
        } else {
            Sv[((size_t)3 * Q + mm) * r + col] = d;
        }
    }
}

// ---------------------------------------------------------------------------
// M2L, kRB columns: one kernel value per node pair serves 4 kRB products, and
// every source value read from LDS serves kNTB target nodes of the thread.
// Threads: kNTB target nodes x a part of the source nodes; parts summed in LDS,
// one field at a time.
// ---------------------------------------------------------------------------
constexpr int kM2LThreadsB = 256;
constexpr int kNTB = 3;

template <typename T, int kRB>
__global__ __launch_bounds__(kM2LThreadsB) void k_m2l_b(DevOp o, int r, const M2LWork *work, const int32_t *partner,
                                                         const double2 *src, double2 *part)
{
    using C = typename dm::cplx_of<T>::type;
    extern __shared__ double smd[];
    const M2LWork wk = work[blockIdx.x];
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    // nodes of the target's level (the partners are on the same level); the cluster
    // arrays keep the stride Qs of the largest degree
    const int Qs = o.Q;
    int lvw = 0;
    while (lvw < o.L && wk.tgt >= o.lvl_off[lvw + 1]) ++lvw;
    const int Q = (o.ql[lvw] + 1) * (o.ql[lvw] + 1);
    const int TPG = (Q + kNTB - 1) / kNTB;
    const int S = max(1, min(kM2LThreadsB / TPG, Q));
    const int SP = (Q + S - 1) / S;
    const int tid = threadIdx.x;
    const int mt = tid % TPG, sp = tid / TPG;
    const bool active = sp < S;
    // node-major staging, so one address (and immediate offsets) reaches a node's data
    T *sX = reinterpret_cast<T *>(smd);                        // [Q][4]: x, y, z, unused
    C *sV = reinterpret_cast<C *>(smd + (4 * Q * (int)sizeof(T) + 15) / 16 * 2);   // [Q][4][kRB], after sX
    double2 *red = reinterpret_cast<double2 *>(smd);           // [S][Q][kRB] (one field at a time)
    __shared__ double2 sTab[256];                               // (cos, sin)(j pi/128), FP64 only
    if constexpr (sizeof(T) == 8)
        for (int i = tid; i < 256; i += kM2LThreadsB) sTab[i] = o.sctab[i];   // first use after a barrier
    const T kap = (T)o.kappa;
    const double *Xt = o.nodeX + (size_t)wk.tgt * 3 * Qs;
    T xt[kNTB][3];
    bool val[kNTB];
#pragma unroll
    for (int t = 0; t < kNTB; ++t) {
        const int mm = mt + t * TPG;
        val[t] = active && mm < Q;
        const int mc = val[t] ? mm : 0;
        xt[t][0] = (T)Xt[mc];
        xt[t][1] = (T)Xt[Qs + mc];
        xt[t][2] = (T)Xt[2 * Qs + mc];
    }
    C acc[kNTB][4][kRB];
#pragma unroll
    for (int t = 0; t < kNTB; ++t)
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int c = 0; c < kRB; ++c) acc[t][f][c] = C{0, 0};
    const int mb = min(Q, sp * SP), me = min(Q, mb + SP);
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const int sc = partner[kp];
        __syncthreads();
        const double *Xs = o.nodeX + (size_t)sc * 3 * Qs;
        const double2 *Vs = src + (size_t)sc * 4 * Qs * r;
        for (int i = tid; i < 3 * Q; i += kM2LThreadsB) sX[(i % Q) * 4 + i / Q] = (T)Xs[(i / Q) * Qs + i % Q];
        for (int i = tid; i < 4 * Q * kRB; i += kM2LThreadsB) {
            const int c = i % kRB, fm = i / kRB, f = fm / Q, m = fm % Q;
            sV[((size_t)m * 4 + f) * kRB + c] = c < nc ? dm::to_c(Vs[((size_t)f * Qs + m) * r + c0 + c], T(0)) : C{0, 0};
        }
        __syncthreads();
        if (active) {
            for (int ms = mb; ms < me; ++ms) {
                const T x0 = sX[4 * ms], x1 = sX[4 * ms + 1], x2 = sX[4 * ms + 2];
                C G[kNTB];
#pragma unroll
                for (int t = 0; t < kNTB; ++t) {
                    const T d0 = xt[t][0] - x0, d1 = xt[t][1] - x1, d2 = xt[t][2] - x2;
                    if constexpr (sizeof(T) == 8) G[t] = dm::helmholtz_r2_tab(kap, fma(d0, d0, fma(d1, d1, d2 * d2)), sTab);
                    else G[t] = dm::helmholtz_r2(kap, fma(d0, d0, fma(d1, d1, d2 * d2)));
                }
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const C *vf = sV + ((size_t)ms * 4 + f) * kRB;
#pragma unroll
                    for (int c = 0; c < kRB; ++c) {
                        const C v = vf[c];
#pragma unroll
                        for (int t = 0; t < kNTB; ++t) acc[t][f][c] = dm::cmac(acc[t][f][c], G[t], v);
                    }
                }
            }
        }
    }
    for (int f = 0; f < 4; ++f) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kNTB; ++t)
            if (val[t])
#pragma unroll
                for (int c = 0; c < kRB; ++c) red[((size_t)sp * Q + mt + t * TPG) * kRB + c] = dm::to_d(acc[t][f][c]);
        __syncthreads();
        for (int i = tid; i < Q * kRB; i += kM2LThreadsB) {
            const int c = i % kRB, mm = i / kRB;
            if (c >= nc) continue;
            double2 v = make_double2(0, 0);
            for (int q2 = 0; q2 < S; ++q2) v = caddb(v, red[((size_t)q2 * Q + mm) * kRB + c]);
            part[(((size_t)blockIdx.x * 4 + f) * Qs + mm) * r + c0 + c] = v;
        }
    }
}

__device__ inline double2 to_d2(double2 v) { return v; }
__device__ inline double2 to_d2(float2 v) { return make_double2(v.x, v.y); }

template <typename PT>
__global__ void k_m2l_reduce_b(DevOp o, int r, const int32_t *wrk_of_tgt, const PT *part, double2 *loc)
{
    const int gc = blockIdx.x, Qs = o.Q;
    int lvl = 0;
    while (lvl < o.L && gc >= o.lvl_off[lvl + 1]) ++lvl;
    const int Q = (o.ql[lvl] + 1) * (o.ql[lvl] + 1);   // nodes of the level (stride Qs)
    const int b = wrk_of_tgt[gc], e = wrk_of_tgt[gc + 1];
    const double ik2 = 1.0 / (o.kappa * o.kappa);
    for (int t = threadIdx.x; t < Q * r; t += blockDim.x) {
        const int mm = t / r, c = t % r;
        double2 u[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
        for (int w = b; w < e; ++w)
            for (int k = 0; k < 4; ++k) u[k] = caddb(u[k], to_d2(part[(((size_t)w * 4 + k) * Qs + mm) * r + c]));
        const double *T = o.nodeT + (size_t)gc * 6 * Qs;
        double2 t1 = make_double2(0, 0), t2 = make_double2(0, 0);
        for (int k = 0; k < 3; ++k) {
            t1 = caddb(t1, cscaleb(T[k * Qs + mm], u[k]));
            t2 = caddb(t2, cscaleb(T[(3 + k) * Qs + mm], u[k]));
        }
        double2 *L = loc + (size_t)gc * 3 * Qs * r;
        if (o.scalar) {   // scalar: |J(x_m)| u (the target's surface element)
            const double Fu[3] = {T[mm], T[Qs + mm], T[2 * Qs + mm]}, Fv[3] = {T[3 * Qs + mm], T[4 * Qs + mm], T[5 * Qs + mm]};
            L[((size_t)0 * Qs + mm) * r + c] = make_double2(0, 0);
            L[((size_t)1 * Qs + mm) * r + c] = make_double2(0, 0);
            L[((size_t)2 * Qs + mm) * r + c] = cscaleb(dm::surf_elem(Fu, Fv), u[3]);
            continue;
        }
        L[((size_t)0 * Qs + mm) * r + c] = t1;
        L[((size_t)1 * Qs + mm) * r + c] = t2;
        L[((size_t)2 * Qs + mm) * r + c] = cscaleb(-ik2, u[3]);
    }
}

// Levels of a smaller degree q_l, kRB columns: source fields at the level's nodes from
// the exact restriction m_l = (R_l (x) R_l)^T m of the degree-q moments
// (R_l[n][m] = L^{q_l}_m(x^q_n)), and local expansions back through R_l (x) R_l.
template <int kRB>
__global__ __launch_bounds__(256) void k_restrict_b(DevOp o, int lvl, int r, const double2 *mom, double2 *src)
{
    extern __shared__ double2 sm2[];
    const int gc = (int)o.lvl_off[lvl] + blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int Q1h = o.Q1, Qs = o.Q, Q1l = o.ql[lvl] + 1, Ql = Q1l * Q1l;
    const double *R = o.Rl + (size_t)lvl * Q1h * Q1h;   // [n][m], m < Q1l
    double2 *M = sm2;                       // [3][Qs][kRB]
    double2 *Z = M + 3 * Qs * kRB;          // [3][Q1h (n2)][Q1l (m1)][kRB]
    const double2 *Mg = mom + (size_t)gc * 3 * Qs * r;
    for (int i = threadIdx.x; i < 3 * Qs * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB;
        M[i] = c < nc ? Mg[(size_t)t * r + c0 + c] : make_double2(0, 0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Q1h * Q1l * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, f = t / (Q1h * Q1l), rm = t % (Q1h * Q1l), n2 = rm / Q1l, m1 = rm % Q1l;
        double2 z = make_double2(0, 0);
        for (int n1 = 0; n1 < Q1h; ++n1) z = caddb(z, cscaleb(R[n1 * Q1h + m1], M[(f * Qs + n2 * Q1h + n1) * kRB + c]));
        Z[i] = z;
    }
    __syncthreads();
    const double *T = o.nodeT + (size_t)gc * 6 * Qs;
    double2 *Sv = src + (size_t)gc * 4 * Qs * r;
    for (int i = threadIdx.x; i < Ql * kRB; i += blockDim.x) {
        const int c = i % kRB, mm = i / kRB, m2 = mm / Q1l, m1 = mm % Q1l;
        if (c >= nc) continue;
        double2 sf[3];
        for (int f = 0; f < 3; ++f) {
            double2 v = make_double2(0, 0);
            for (int n2 = 0; n2 < Q1h; ++n2)
                v = caddb(v, cscaleb(R[n2 * Q1h + m2], Z[((f * Q1h + n2) * Q1l + m1) * kRB + c]));
            sf[f] = v;
        }
        const double Fu[3] = {T[mm], T[Qs + mm], T[2 * Qs + mm]}, Fv[3] = {T[3 * Qs + mm], T[4 * Qs + mm], T[5 * Qs + mm]};
        const size_t col = c0 + c;
        if (o.scalar) {
            for (int k = 0; k < 3; ++k) Sv[((size_t)k * Qs + mm) * r + col] = make_double2(0, 0);
            Sv[((size_t)3 * Qs + mm) * r + col] = cscaleb(dm::surf_elem(Fu, Fv), sf[2]);
        } else {
            for (int k = 0; k < 3; ++k)
                Sv[((size_t)k * Qs + mm) * r + col] = caddb(cscaleb(Fu[k], sf[0]), cscaleb(Fv[k], sf[1]));
            Sv[((size_t)3 * Qs + mm) * r + col] = sf[2];
        }
    }
}

template <int kRB>
__global__ __launch_bounds__(256) void k_lift_b(DevOp o, int lvl, int r, double2 *loc)
{
    extern __shared__ double2 sm2[];
    const int gc = (int)o.lvl_off[lvl] + blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int Q1h = o.Q1, Qs = o.Q, Q1l = o.ql[lvl] + 1, Ql = Q1l * Q1l;
    const double *R = o.Rl + (size_t)lvl * Q1h * Q1h;
    double2 *A = sm2;                       // [3][Ql][kRB]
    double2 *Y = A + 3 * Ql * kRB;          // [3][Q1l (m2)][Q1h (n1)][kRB]
    double2 *Lc = loc + (size_t)gc * 3 * Qs * r;
    for (int i = threadIdx.x; i < 3 * Ql * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB;
        A[i] = c < nc ? Lc[((size_t)(t / Ql) * Qs + t % Ql) * r + c0 + c] : make_double2(0, 0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Q1l * Q1h * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, f = t / (Q1l * Q1h), rm = t % (Q1l * Q1h), m2 = rm / Q1h, n1 = rm % Q1h;
        double2 y = make_double2(0, 0);
        for (int m1 = 0; m1 < Q1l; ++m1) y = caddb(y, cscaleb(R[n1 * Q1h + m1], A[(f * Ql + m2 * Q1l + m1) * kRB + c]));
        Y[i] = y;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Qs * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, f = t / Qs, nn = t % Qs, n2 = nn / Q1h, n1 = nn % Q1h;
        if (c >= nc) continue;
        double2 v = make_double2(0, 0);
        for (int m2 = 0; m2 < Q1l; ++m2) v = caddb(v, cscaleb(R[n2 * Q1h + m2], Y[((f * Q1l + m2) * Q1h + n1) * kRB + c]));
        Lc[(size_t)t * r + c0 + c] = v;
    }
}

template <int kRB>
__global__ __launch_bounds__(256) void k_l2l_b(DevOp o, int lvl, int r, double2 *loc)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int S = 1 << lvl, Q1 = o.Q1, Q = o.Q;
    const int j = id / (S * S), rr = id % (S * S), k2 = rr / S, k1 = rr % S;
    const int gc = (int)o.lvl_off[lvl] + id;
    const int Sp = S / 2;
    const int pgc = (int)o.lvl_off[lvl - 1] + (j * Sp + k2 / 2) * Sp + k1 / 2;
    const int c1 = k1 & 1, c2 = k2 & 1;
    const double *Tu = c1 ? o.T1 : o.T0, *Tv = c2 ? o.T1 : o.T0;
    const double2 *par = loc + (size_t)pgc * 3 * Q * r;
    double2 *W = sm2;                 // [3][Q1 (m2)][Q1 (n1)][kRB]
    double2 *X = W + 3 * Q * kRB;     // the parent's fields, staged once (coalesced along columns)
    for (int i = threadIdx.x; i < 3 * Q * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB;
        X[i] = c < nc ? par[(size_t)t * r + c0 + c] : make_double2(0, 0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Q * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, f = t / Q, rem = t % Q, m2 = rem / Q1, n1 = rem % Q1;
        double2 z = make_double2(0, 0);
        for (int m1 = 0; m1 < Q1; ++m1) z = caddb(z, cscaleb(Tu[n1 * Q1 + m1], X[((f * Q) + m2 * Q1 + m1) * kRB + c]));
        W[i] = z;
    }
    __syncthreads();
    double2 *chd = loc + (size_t)gc * 3 * Q * r;
    for (int i = threadIdx.x; i < 3 * Q * kRB; i += blockDim.x) {
        const int c = i % kRB, t = i / kRB, f = t / Q, rem = t % Q, n2 = rem / Q1, n1 = rem % Q1;
        if (c >= nc) continue;
        double2 z = chd[((size_t)f * Q + rem) * r + c0 + c];
        for (int m2 = 0; m2 < Q1; ++m2) z = caddb(z, cscaleb(Tv[n2 * Q1 + m2], W[((f * Q) + m2 * Q1 + n1) * kRB + c]));
        chd[((size_t)f * Q + rem) * r + c0 + c] = z;
    }
}

template <int kRB>
__global__ __launch_bounds__(256) void k_l2p_leaf_b(DevOp o, int r, const double2 *loc, double2 *ybuf)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen;
    const int rr = id % (SL * SL), k2 = rr / SL, k1 = rr % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    const double2 *t = loc + (size_t)gc * 3 * Q * r;
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mqu = o.Mq + (size_t)k1 * Q1 * RL, *Mdu = o.Mdp + (size_t)k1 * Q1 * RL;
    const double *Mpv = o.Mp + (size_t)k2 * Q1 * RL, *Mqv = o.Mq + (size_t)k2 * Q1 * RL, *Mdv = o.Mdp + (size_t)k2 * Q1 * RL;
    double2 *W0 = sm2;                    // [Q1][RL][kRB]
    double2 *W1 = W0 + Q1 * RL * kRB;
    double2 *W1d = W1 + Q1 * RL * kRB;
    double2 *T3 = W1d + Q1 * RL * kRB;    // the leaf's three fields [3][Q][kRB], read once
    const int w1a = s + p, w1b = s + p - 1;
    for (int i = threadIdx.x; i < 3 * Q * kRB; i += blockDim.x) {
        const int c = i % kRB, tt = i / kRB;
        T3[i] = c < nc ? t[(size_t)tt * r + c0 + c] : make_double2(0, 0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Q1 * RL * kRB; i += blockDim.x) {
        const int c = i % kRB, tt = i / kRB, m2 = tt / RL, i1 = tt % RL;
        double2 a = make_double2(0, 0), b = make_double2(0, 0), bd = make_double2(0, 0);
        if (c < nc)
            for (int m1 = 0; m1 < Q1; ++m1) {
                const double2 f1 = T3[((0 * Q + m2 * Q1 + m1)) * kRB + c];
                const double2 f2 = T3[((1 * Q + m2 * Q1 + m1)) * kRB + c];
                const double2 fd = T3[((2 * Q + m2 * Q1 + m1)) * kRB + c];
                if (i1 < w1a) a = caddb(a, caddb(cscaleb(Mpu[m1 * RL + i1], f1), cscaleb(Mdu[m1 * RL + i1], fd)));
                if (i1 < w1b) {
                    b = caddb(b, cscaleb(Mqu[m1 * RL + i1], f2));
                    bd = caddb(bd, cscaleb(Mqu[m1 * RL + i1], fd));
                }
            }
        W0[i] = a;
        W1[i] = b;
        W1d[i] = bd;
    }
    __syncthreads();
    double2 *Y = ybuf + (size_t)id * 2 * RL * RL * r;
    for (int i = threadIdx.x; i < 2 * RL * RL * kRB; i += blockDim.x) {
        const int c = i % kRB, tt = i / kRB, ch = tt / (RL * RL), rem = tt % (RL * RL), i2 = rem / RL, i1 = rem % RL;
        if (c >= nc) continue;
        double2 v = make_double2(0, 0);
        if (ch == 0 && i2 < s + p - 1 && i1 < w1a) {
            for (int m2 = 0; m2 < Q1; ++m2) v = caddb(v, cscaleb(Mqv[m2 * RL + i2], W0[(m2 * RL + i1) * kRB + c]));
        } else if (ch == 1 && i2 < s + p && i1 < w1b) {
            for (int m2 = 0; m2 < Q1; ++m2)
                v = caddb(v, caddb(cscaleb(Mpv[m2 * RL + i2], W1[(m2 * RL + i1) * kRB + c]),
                                   cscaleb(Mdv[m2 * RL + i2], W1d[(m2 * RL + i1) * kRB + c])));
        }
        Y[(size_t)tt * r + c0 + c] = v;
    }
}

// scalar single layer, kRB columns: Y[i2][i1] = sum (M_p (x) M_p)^T t^d over the
// leaf's W x W window (channel 0 of the leaf's result rows; channel 1 zero)
template <int kRB>
__global__ __launch_bounds__(256) void k_l2p_leaf_sc_b(DevOp o, int r, const double2 *loc, double2 *ybuf)
{
    extern __shared__ double2 sm2[];
    const int id = blockIdx.x;
    const int c0 = blockIdx.y * kRB, nc = min(kRB, r - c0);
    const int SL = o.SL, s = o.s, p = o.p, Q1 = o.Q1, Q = o.Q, RL = o.rowlen, W = s + p;
    const int rr = id % (SL * SL), k2 = rr / SL, k1 = rr % SL;
    const int gc = (int)o.lvl_off[o.L] + id;
    const double2 *t = loc + ((size_t)gc * 3 + 2) * Q * r;
    const double *Mpu = o.Mp + (size_t)k1 * Q1 * RL, *Mpv = o.Mp + (size_t)k2 * Q1 * RL;
    double2 *Wm = sm2;                    // [Q1 (m2)][W (i1)][kRB]
    double2 *Td = Wm + Q1 * W * kRB;      // the leaf's field [Q][kRB], read once
    for (int i = threadIdx.x; i < Q * kRB; i += blockDim.x) {
        const int c = i % kRB, tt = i / kRB;
        Td[i] = c < nc ? t[(size_t)tt * r + c0 + c] : make_double2(0, 0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Q1 * W * kRB; i += blockDim.x) {
        const int c = i % kRB, tt = i / kRB, m2 = tt / W, i1 = tt % W;
        double2 a = make_double2(0, 0);
        if (c < nc)
            for (int m1 = 0; m1 < Q1; ++m1) a = caddb(a, cscaleb(Mpu[m1 * RL + i1], Td[(m2 * Q1 + m1) * kRB + c]));
        Wm[i] = a;
    }
    __syncthreads();
    double2 *Y = ybuf + (size_t)id * 2 * RL * RL * r;
    for (int i = threadIdx.x; i < 2 * RL * RL * kRB; i += blockDim.x) {
        const int c = i % kRB, tt = i / kRB, ch = tt / (RL * RL), rem = tt % (RL * RL), i2 = rem / RL, i1 = rem % RL;
        if (c >= nc) continue;
        double2 v = make_double2(0, 0);
        if (ch == 0 && i2 < W && i1 < W)
            for (int m2 = 0; m2 < Q1; ++m2) v = caddb(v, cscaleb(Mpv[m2 * RL + i2], Wm[(m2 * W + i1) * kRB + c]));
        Y[(size_t)tt * r + c0 + c] = v;
    }
}

__global__ void k_l2p_gather_b(DevOp o, int r, const double2 *ybuf, double2 *yt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)o.N * r) return;
    const int i = (int)(t / r), col = (int)(t % r);
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
                const double2 v = ybuf[((((size_t)leaf * 2 + a) * RL + (i2 - k2 * s)) * RL + (i1 - k1 * s)) * r + col];
                acc = caddb(acc, cscaleb(sg, v));
            }
    }
    yt[t] = caddb(yt[t], acc);
}

}  // namespace

// ---------------------------------------------------------------------------
// batched apply: y = A x for r columns (x, y: [r][N] device); xt, yt: [N][r]
// scratch; the operator's batched workspaces must hold r columns.
// Each kernel takes the largest column chunk (8, 4, 2, 1) whose LDS fits 64 KB.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kLdsMax = 64 * 1024;

// columns per workgroup: the most that fit a shared-memory budget.  The transfer
// kernels (P2M, M2M, L2L, L2P) take a 32 KB budget by default (IGE_BATCH_LDS_KB): more,
// smaller workgroups hide their latency better (level 6, 64 columns: 0.64 -> 0.53 ms
// for the four); the generated coupling keeps 64 KB.
size_t transfer_lds()
{
    static const size_t lds = [] {
        const char *e = std::getenv("IGE_BATCH_LDS_KB");
        return e ? std::min(kLdsMax, (size_t)std::max(1, std::atoi(e)) * 1024) : (size_t)32 * 1024;
    }();
    return lds;
}

int pick_rb(size_t bytes_per_col, size_t fixed = 0, size_t budget = transfer_lds())
{
    for (int rb = kRBMax; rb > 1; rb /= 2)
        if (fixed + bytes_per_col * rb <= budget) return rb;
    return 1;
}
}  // namespace

namespace {
// [r][N] <-> [N][r]: tiled for 16 columns or more, direct below (a tile would be
// mostly empty)
void transpose_cols(hipStream_t s, int64_t N, int r, const double2 *in, double2 *out, bool to_rows)
{
    const int64_t tot = N * r;
    if (r >= 16) {
        const dim3 grid((unsigned)((N + kTT - 1) / kTT), (unsigned)((r + kTT - 1) / kTT));
        if (to_rows) hipLaunchKernelGGL(k_transpose_t<true>, grid, dim3(256), 0, s, N, r, in, out);
        else hipLaunchKernelGGL(k_transpose_t<false>, grid, dim3(256), 0, s, N, r, in, out);
    } else if (to_rows) {
        hipLaunchKernelGGL(k_to_rows, dim3((tot + 255) / 256), dim3(256), 0, s, N, r, in, out);
    } else {
        hipLaunchKernelGGL(k_to_cols, dim3((tot + 255) / 256), dim3(256), 0, s, N, r, in, out);
    }
    IGE_HIP(hipGetLastError());
}
}  // namespace

#define IGE_RB_SWITCH(rb, KERNEL, grid, block, shm, stream, ...)                                             \
    switch (rb) {                                                                                            \
        case 8: hipLaunchKernelGGL(KERNEL<8>, grid, block, shm, stream, __VA_ARGS__); break;                \
        case 4: hipLaunchKernelGGL(KERNEL<4>, grid, block, shm, stream, __VA_ARGS__); break;                \
        case 2: hipLaunchKernelGGL(KERNEL<2>, grid, block, shm, stream, __VA_ARGS__); break;                \
        default: hipLaunchKernelGGL(KERNEL<1>, grid, block, shm, stream, __VA_ARGS__); break;               \
    }                                                                                                        \
    IGE_HIP(hipGetLastError())

int near_mfma_mtw_ok(int nF, int rc);
void near_batched_mfma(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s);

void apply_batched(ige_op op, int r, const double2 *x, double2 *y, double2 *xt, double2 *yt, hipEvent_t *ev, int prec)
{
    const DevOp &o = op->view;
    hipStream_t s = lstream(op);
    auto mark_on = [&](int i, hipStream_t st) {
        if (ev && prof_records(op, i)) IGE_HIP(hipEventRecord(ev[i], st));
    };
    auto mark = [&](int i) { mark_on(i, s); };
    const int64_t N = o.N;
    const int64_t tot = N * r;
    auto chunks = [&](int rb) { return (r + rb - 1) / rb; };
    if (x) {   // x == nullptr: xt already holds the input (graph body)
        transpose_cols(s, N, r, x, xt, true);
    }
    const bool far = !op->work.empty();
    // the near-field product on the operator's second stream beside the far field,
    // joined before the gather (batch_overlap 1: from the start, 2: after M2M)
    const int ovl = far && op->overlap ? op->batch_overlap : 0;
    hipStream_t s2 = op->aux;
    auto near = [&](hipStream_t st) {
        mark_on(7, st);
        if (prec == IGE_BF16X3_ALL) near_bf16(op, r, xt, yt, st);
        else if (near_f64mx_ok(op, r)) near_f64mx(op, r, xt, yt, st);
        else if (r >= 8 && near_mfma_mtw_ok(o.nF, o.rc)) near_batched_mfma(op, r, xt, yt, st);
        else near_batched(op, r, xt, yt, st);
        mark_on(11, st);
        mark_on(8, st);
    };
    auto fork_near = [&] {
        IGE_HIP(hipEventRecord(op->ev_fork, s));
        IGE_HIP(hipStreamWaitEvent(s2, op->ev_fork, 0));
        near(s2);
        IGE_HIP(hipEventRecord(op->ev_join, s2));
    };
    if (ovl == 1) fork_near();
    mark(0);
    if (far) {
        const int nleaf = o.P * o.SL * o.SL;
        const size_t w1a = o.s + o.p;
        if (o.scalar) {
            const size_t per = sizeof(double2) * (w1a * w1a + w1a * o.Q1);
            const int rb = pick_rb(per);
            IGE_RB_SWITCH(rb, k_p2m_sc_b, dim3(nleaf, chunks(rb)), dim3(256), per * rb, s, o, r, xt, op->d_bmom.p,
                          op->d_bsrc.p);
        } else {
            const size_t per = sizeof(double2) * (2 * w1a * w1a + 3 * w1a * o.Q1);
            const int rb = pick_rb(per);
            IGE_RB_SWITCH(rb, k_p2m_b, dim3(nleaf, chunks(rb)), dim3(256), per * rb, s, o, r, xt, op->d_bmom.p,
                          op->d_bsrc.p);
        }
        mark(1);
        {
            const size_t per = sizeof(double2) * 9 * o.Q;   // accumulators, intermediate, staged child (3 fields each)
            const int rb = pick_rb(per);
            for (int lvl = o.L - 1; lvl >= std::max(0, op->lfar); --lvl) {   // as the single-column pass
                IGE_RB_SWITCH(rb, k_m2m_b, dim3(o.P << (2 * lvl), chunks(rb)), dim3(256), per * rb, s, o, lvl, r,
                              op->d_bmom.p, op->d_bsrc.p);
            }
        }
        if (o.varq)   // levels of a smaller degree: source fields from the restricted moments
            for (int lvl = std::max(0, op->lfar); lvl <= o.L; ++lvl) {
                const size_t Q1l = o.ql[lvl] + 1;
                if ((int)Q1l == o.Q1) continue;
                const size_t per = sizeof(double2) * (3 * (size_t)o.Q + 3 * (size_t)o.Q1 * Q1l);
                const int rb = pick_rb(per);
                IGE_RB_SWITCH(rb, k_restrict_b, dim3(o.P << (2 * lvl), chunks(rb)), dim3(256), per * rb, s, o, lvl, r,
                              op->d_bmom.p, op->d_bsrc.p);
            }
        mark(2);
        if (ovl == 2) fork_near();
        if (prec == IGE_BF16 || prec == IGE_BF16X3 || prec == IGE_BF16X3_ALL) {
            m2l_bf16(op, r, prec == IGE_BF16 ? 1 : 3, op->d_bsrc.p, s, ev ? ev[12] : nullptr);
            mark(3);
            hipLaunchKernelGGL(k_m2l_reduce_b<float2>, dim3(op->NC), dim3(256), 0, s, o, r, op->d_mwrk_of_tgt.p,
                               op->d_bmpart.p, op->d_bloc.p);
            IGE_HIP(hipGetLastError());
        } else if (prec == IGE_F64 && m2l_f64mx_use(op, r)) {
            m2l_f64mx(op, r, op->d_bsrc.p, s, ev ? ev[12] : nullptr);
            mark(3);
            hipLaunchKernelGGL(k_m2l_reduce_b<double2>, dim3(op->NC), dim3(256), 0, s, o, r, op->d_mwrk_of_tgt.p,
                               op->d_bmpart64.p, op->d_bloc.p);
            IGE_HIP(hipGetLastError());
        } else if (op->stored) {
            mark(12);
            m2l_stored(op, r, prec, op->d_bsrc.p, op->d_bloc.p, s);
            mark(3);
        } else {
            mark(12);
            {
                // shared memory for the largest of the levels' node counts
                size_t per = 0;
                for (int lvl = std::max(0, op->lfar); lvl <= o.L; ++lvl) {
                    const int Ql = (o.ql[lvl] + 1) * (o.ql[lvl] + 1);
                    const int TPG = (Ql + kNTB - 1) / kNTB;
                    const int S = std::max(1, std::min(kM2LThreadsB / TPG, Ql));
                    per = std::max(per, std::max(sizeof(double2) * 4 * Ql, sizeof(double2) * (size_t)S * Ql));
                }
                const size_t fixed = sizeof(double) * 4 * o.Q;
                // registers: 3 targets x 4 fields x rb columns; a tuned value may only lower it
                const int rbmax = std::min(4, pick_rb(per, fixed, kLdsMax));
                const int rb = std::min(rbmax, tune_get(op, kTuneM2lRb, r, prec, rbmax));
                const dim3 grid(op->work.size(), chunks(rb)), blk(kM2LThreadsB);
                const size_t shm = fixed + per * rb;
                if (prec == IGE_F32) {
                    switch (rb) {
                        case 4: hipLaunchKernelGGL((k_m2l_b<float, 4>), grid, blk, shm, s, o, r, op->d_work.p, op->d_partner.p, op->d_bsrc.p, op->d_bpart.p); break;
                        case 2: hipLaunchKernelGGL((k_m2l_b<float, 2>), grid, blk, shm, s, o, r, op->d_work.p, op->d_partner.p, op->d_bsrc.p, op->d_bpart.p); break;
                        default: hipLaunchKernelGGL((k_m2l_b<float, 1>), grid, blk, shm, s, o, r, op->d_work.p, op->d_partner.p, op->d_bsrc.p, op->d_bpart.p); break;
                    }
                } else {
                    switch (rb) {
                        case 4: hipLaunchKernelGGL((k_m2l_b<double, 4>), grid, blk, shm, s, o, r, op->d_work.p, op->d_partner.p, op->d_bsrc.p, op->d_bpart.p); break;
                        case 2: hipLaunchKernelGGL((k_m2l_b<double, 2>), grid, blk, shm, s, o, r, op->d_work.p, op->d_partner.p, op->d_bsrc.p, op->d_bpart.p); break;
                        default: hipLaunchKernelGGL((k_m2l_b<double, 1>), grid, blk, shm, s, o, r, op->d_work.p, op->d_partner.p, op->d_bsrc.p, op->d_bpart.p); break;
                    }
                }
                IGE_HIP(hipGetLastError());
            }
            mark(3);
            hipLaunchKernelGGL(k_m2l_reduce_b<double2>, dim3(op->NC), dim3(256), 0, s, o, r, op->d_wrk_of_tgt.p, op->d_bpart.p,
                               op->d_bloc.p);
            IGE_HIP(hipGetLastError());
        }
        if (o.varq)   // levels of a smaller degree: local expansions back to the degree-q nodes
            for (int lvl = std::max(0, op->lfar); lvl <= o.L; ++lvl) {
                const size_t Q1l = o.ql[lvl] + 1;
                if ((int)Q1l == o.Q1) continue;
                const size_t per = sizeof(double2) * (3 * Q1l * Q1l + 3 * Q1l * (size_t)o.Q1);
                const int rb = pick_rb(per);
                IGE_RB_SWITCH(rb, k_lift_b, dim3(o.P << (2 * lvl), chunks(rb)), dim3(256), per * rb, s, o, lvl, r,
                              op->d_bloc.p);
            }
        mark(4);
        {
            const size_t per = sizeof(double2) * 6 * o.Q;   // intermediate and staged parent
            const int rb = pick_rb(per);
            for (int lvl = std::max(1, op->lfar + 1); lvl <= o.L; ++lvl) {
                IGE_RB_SWITCH(rb, k_l2l_b, dim3(o.P << (2 * lvl), chunks(rb)), dim3(256), per * rb, s, o, lvl, r,
                              op->d_bloc.p);
            }
        }
        mark(5);
        if (o.scalar) {
            const size_t per = sizeof(double2) * ((size_t)o.Q1 * w1a + (size_t)o.Q);
            const int rb = pick_rb(per, 0, kLdsMax);
            IGE_RB_SWITCH(rb, k_l2p_leaf_sc_b, dim3(nleaf, chunks(rb)), dim3(256), per * rb, s, o, r, op->d_bloc.p,
                          op->d_bybuf.p);
        } else {   // three intermediates and the staged fields
            const size_t per = sizeof(double2) * (3 * (size_t)o.Q1 * o.rowlen + 3 * (size_t)o.Q);
            const int rb = pick_rb(per, 0, kLdsMax);
            IGE_RB_SWITCH(rb, k_l2p_leaf_b, dim3(nleaf, chunks(rb)), dim3(256), per * rb, s, o, r, op->d_bloc.p,
                          op->d_bybuf.p);
        }
        mark(6);
    } else {
        for (int i = 1; i <= 6; ++i) mark(i);
        mark(12);
    }
    if (ovl) IGE_HIP(hipStreamWaitEvent(s, op->ev_join, 0));
    else near(s);
    mark(9);
    if (far) {
        hipLaunchKernelGGL(k_l2p_gather_b, dim3((tot + 255) / 256), dim3(256), 0, s, o, r, op->d_bybuf.p, yt);
        IGE_HIP(hipGetLastError());
    }
    mark(10);
    if (y) {   // y == nullptr: the result stays in yt (graph body)
        transpose_cols(s, N, r, yt, y, false);
    }
}

void batched_to_rows(ige_op op, int r, const double2 *x, double2 *xt, hipStream_t s)
{
    transpose_cols(s, (int64_t)op->view.N, r, x, xt, true);
}

void batched_to_cols(ige_op op, int r, const double2 *yt, double2 *y, hipStream_t s)
{
    transpose_cols(s, (int64_t)op->view.N, r, yt, y, false);
}

}  // namespace ige

// ---------------------------------------------------------------------------
// Near-field product for many columns on the FP64 matrix cores (16x16x4: lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; accumulator register j of lane l holds
// D[l/16 + 4j][l%16]).  For a stored block B (target leaf t, source leaf s) and the
// row chunk [r0, r0 + rc):
//   DIR 0: Y_t[r0 + m][n] = sum_k B[r0 + m][k] X_s[k][n]            (rows of the chunk)
//   DIR 1: Y_s[m][n]      = sum_{k < rc} B[r0 + k][m] X_t[r0 + k][n]  (off-diagonal blocks)
// Complex products as four real ones: Yr += Br Xr - Bi Xi, Yi += Br Xi + Bi Xr.
// A workgroup takes one (block, row chunk) and 16 NT columns; wave w owns the column
// tile w % NT and every (4 / NT)-th row tile.  Results go to the partial-result slots
// ([slot][r]) that the fixed-order per-unknown reduction sums.
// ---------------------------------------------------------------------------
namespace ige {
namespace {

typedef double dx4b __attribute__((ext_vector_type(4)));

constexpr int kNearMfmaMaxK = 1024;   // reduction length staged in shared memory (slots per leaf)
constexpr int kNearMfmaPD = 2;        // reduction steps loaded ahead of the products

template <int DIR, int NT, int MTW>
__global__ __launch_bounds__(256) void k_near_mfma(DevOp o, int r, const double2 *xt, double2 *part)
{
    __shared__ int32_t skd[kNearMfmaMaxK];   // unknown of every reduction index (-1: none)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nF = o.nF;
    const int64_t b = blockIdx.x / o.nch;
    const int ch = blockIdx.x % o.nch;
    const int lt = o.bpair[2 * b], ls = o.bpair[2 * b + 1];
    if (DIR == 1 && lt == ls) return;   // diagonal blocks: no transposed product
    const int r0 = ch * o.rc, rc = min(o.rc, nF - r0);
    const int c0 = blockIdx.y * 16 * NT;
    const int M = DIR == 0 ? rc : nF, K = DIR == 0 ? nF : rc;
    const int MT = (M + 15) / 16, KS = (K + 3) / 4;
    const int nt = wv % NT, mstep = 4 / NT, mfirst = wv / NT;
    const int n = c0 + 16 * nt + (lane & 15);   // this lane's column (B operand and output)
    const bool nok = n < r;
    const int nc = nok ? n : 0;
    const double2 *Bv = o.bval + (size_t)b * nF * nF;
    const int32_t *kdof = o.leafdof + (size_t)(DIR == 0 ? ls : lt) * nF + (DIR == 0 ? 0 : r0);
    for (int i = threadIdx.x; i < K; i += blockDim.x) skd[i] = kdof[i];
    __syncthreads();
    dx4b accr[MTW], acci[MTW];
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
        accr[i] = dx4b{0.0, 0.0, 0.0, 0.0};
        acci[i] = dx4b{0.0, 0.0, 0.0, 0.0};
    }
    // operands of reduction step s: every load from a clamped, valid address, zeroed
    // where out of range (no branches around the loads, so they stay in flight)
    auto load = [&](int s, double2 &xo, double2 (&ao)[MTW]) {
        const int k = 4 * s + (lane >> 4);   // reduction index supplied by this lane
        const int d = (k < K && nok) ? skd[min(k, K - 1)] : -1;
        const double2 v = xt[(size_t)max(d, 0) * r + nc];
        xo = d >= 0 ? v : make_double2(0.0, 0.0);
        const int ka = min(k, K - 1);
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
            const int mt = mfirst + i * mstep;
            if (mt < MT) {   // uniform over the wave
                const int m = 16 * mt + (lane & 15), mc = min(m, M - 1);
                const double2 av = DIR == 0 ? Bv[(size_t)(r0 + mc) * nF + ka] : Bv[(size_t)(r0 + ka) * nF + mc];
                ao[i] = (m < M && k < K) ? av : make_double2(0.0, 0.0);
            }
        }
    };
    double2 xb[kNearMfmaPD], ab[kNearMfmaPD][MTW];
#pragma unroll
    for (int d = 0; d < kNearMfmaPD; ++d)
        if (d < KS) load(d, xb[d], ab[d]);
    for (int s0 = 0; s0 < KS; s0 += kNearMfmaPD) {
#pragma unroll
        for (int d = 0; d < kNearMfmaPD; ++d) {
            const int s = s0 + d;
            if (s < KS) {   // uniform
                const double xr = xb[d].x, xi = xb[d].y;
                double2 a[MTW];
#pragma unroll
                for (int i = 0; i < MTW; ++i) a[i] = ab[d][i];
                if (s + kNearMfmaPD < KS) load(s + kNearMfmaPD, xb[d], ab[d]);
#pragma unroll
                for (int i = 0; i < MTW; ++i) {
                    if (mfirst + i * mstep < MT) {   // uniform over the wave
                        accr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, xr, accr[i], 0, 0, 0);
                        accr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[i].y, xi, accr[i], 0, 0, 0);
                        acci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, xi, acci[i], 0, 0, 0);
                        acci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, xr, acci[i], 0, 0, 0);
                    }
                }
            }
        }
    }
    if (!nok) return;
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
        const int mt = mfirst + i * mstep;
        if (mt >= MT) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 16 * mt + (lane >> 4) + 4 * j;
            if (m >= M) continue;
            const size_t slot = DIR == 0 ? (size_t)b * nF + r0 + m
                                         : (size_t)o.nblk * nF + ((size_t)b * o.nch + ch) * nF + m;
            part[slot * r + n] = make_double2(accr[i][j], acci[i][j]);
        }
    }
}

// yt[i][c] = sum of the partial results of unknown i, column c ([slot][r] layout),
// 16 lanes per (unknown, column) with a fixed butterfly
__global__ __launch_bounds__(256) void k_near_gather_r(int N, int r, const int64_t *ptr, const int32_t *idx,
                                                       const double2 *part, double2 *yt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sub = (int)(t & 15);
    const int64_t ic = t >> 4;
    const int64_t i = ic / r;
    const int c = (int)(ic % r);
    double re = 0.0, im = 0.0;
    if (i < N)
        for (int64_t k = ptr[i] + sub; k < ptr[i + 1]; k += 16) {
            const double2 v = part[(size_t)idx[k] * r + c];
            re += v.x;
            im += v.y;
        }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off, 16);
        im += __shfl_xor(im, off, 16);
    }
    if (i < N && sub == 0) yt[(size_t)i * r + c] = make_double2(re, im);
}

template <int DIR, int NT>
void launch_near_mfma(ige_op op, int r, const double2 *xt, double2 *part, hipStream_t s)
{
    const DevOp &o = op->view;
    const int M = DIR == 0 ? o.rc : o.nF;
    const int MT = (M + 15) / 16, mstep = 4 / NT;
    const int mtw = (MT + mstep - 1) / mstep;
    const dim3 grid((unsigned)(o.nblk * o.nch), (unsigned)((r + 16 * NT - 1) / (16 * NT))), blk(256);
#define IGE_NM_CASE(W)                                                                                   \
    case W: hipLaunchKernelGGL((k_near_mfma<DIR, NT, W>), grid, blk, 0, s, o, r, xt, part); break;
    switch (mtw) {
        IGE_NM_CASE(1)
        IGE_NM_CASE(2)
        IGE_NM_CASE(3)
        IGE_NM_CASE(4)
        IGE_NM_CASE(6)
        IGE_NM_CASE(8)
        IGE_NM_CASE(12)
        IGE_NM_CASE(16)
        default: throw Status{IGE_EINVAL, "near-field block too large for the matrix-core product"};
    }
#undef IGE_NM_CASE
    IGE_HIP(hipGetLastError());
}

}  // namespace

int near_mfma_mtw_ok(int nF, int rc)
{
    if (nF > kNearMfmaMaxK) return 0;
    for (int NT : {1, 2, 4})
        for (int M : {rc, nF}) {
            const int MT = (M + 15) / 16, ms = 4 / NT, w = (MT + ms - 1) / ms;
            if (w > 16 || (w > 4 && w != 6 && w != 8 && w != 12 && w != 16)) return 0;
        }
    return 1;
}

void near_batched_mfma(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s)
{
    const DevOp &o = op->view;
    const size_t need = (size_t)o.nblk * o.nF * (1 + o.nch) * r;
    if (op->d_bnpart_r.n < need) op->d_bnpart_r.alloc(need);
    double2 *part = op->d_bnpart_r.p;
    const int NT = tune_get(op, kTuneNearMfmaNt, r, 0, r > 16 ? 2 : 1);
    if (NT == 4) {
        launch_near_mfma<0, 4>(op, r, xt, part, s);
        launch_near_mfma<1, 4>(op, r, xt, part, s);
    } else if (NT == 2) {
        launch_near_mfma<0, 2>(op, r, xt, part, s);
        launch_near_mfma<1, 2>(op, r, xt, part, s);
    } else {
        launch_near_mfma<0, 1>(op, r, xt, part, s);
        launch_near_mfma<1, 1>(op, r, xt, part, s);
    }
    const int64_t tot = (int64_t)o.N * r * 16;
    hipLaunchKernelGGL(k_near_gather_r, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, o.N, r, o.red_ptr,
                       o.red_idx, part, yt);
    IGE_HIP(hipGetLastError());
}

}  // namespace ige
