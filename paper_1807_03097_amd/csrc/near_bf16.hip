// Near-field product in split BF16 on the matrix cores, for the inner solves
// of the mixed-precision iterative refinement (the near-field blocks themselves are
// assembled in FP64 by the Galerkin quadrature of Sec. 3; this is a lower-precision
// copy of them for the inner operator only).
//
// Every ordered leaf pair (t, s) of the near field gets its own block
// A_ts = B_b (t = target leaf of the stored block b) or B_b^T (t = its source leaf),
// stored as rows [Re | Im] over the slot index of s, zero padded to Qp (a multiple of
// 32), each entry as a BF16 pair x = xh + xl.  For a target leaf t and its partners s:
//   Y_t = sum_s A_ts X_s,  Yr += Ar Xr - Ai Xi,  Yi += Ai Xr + Ar Xi,
// where each real product runs on the 16x16x32 BF16 instruction as xh.yh + xh.yl +
// xl.yh with FP32 accumulation (about 2^-16 relative).  The right factors X_s are the
// columns of x gathered to the function slots of leaf s (signs of the glued unknowns
// are folded into the blocks).  Work: one workgroup per (target leaf, up to 8
// partners, chunk of 16 NT columns), wave w owning row tiles w MTW .. w MTW + MTW - 1;
// partial results per work item (FP32) are summed per unknown in a fixed order.
//
// The FP64 operator of many columns uses the same ordered-pair blocks in FP64 on the
// FP64 matrix cores (last part of this file): rows [Br, -Bi] and [Bi, Br] read from the
// stored [Br | Bi] as one real product with [Re X; Im X], as in the FP64 coupling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "op.hpp"

namespace ige {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kNearPartners = 8;   // partners per work item

__device__ inline void split_pair(double x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)(float)x;
    lo = (__bf16)(float)(x - (double)(float)hi);
}

__device__ inline bf8 neg8(bf8 x)
{
    uint4 u = __builtin_bit_cast(uint4, x);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(bf8, u);
}

// Ab[2 b + ori][plane][Qp][2 Qp]: ori 0 row i = B_b[i][:], ori 1 row i = B_b[:][i]
__global__ void k_nb_store(const double2 *bval, int64_t nblk, int nF, int Qp, __bf16 *Ab)
{
    const int K2 = 2 * Qp;
    const int64_t per = (int64_t)Qp * Qp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * nblk * per) return;
    const int64_t po = t / per;
    const int rem = (int)(t % per), i = rem / Qp, j = rem % Qp;
    const int64_t b = po / 2;
    const int ori = (int)(po % 2);
    double2 v = make_double2(0.0, 0.0);
    if (i < nF && j < nF) v = ori == 0 ? bval[((size_t)b * nF + i) * nF + j] : bval[((size_t)b * nF + j) * nF + i];
    __bf16 *base = Ab + (size_t)po * 2 * Qp * K2;
    const size_t ire = (size_t)i * K2 + j, iim = ire + Qp;
    __bf16 h, l;
    split_pair(v.x, h, l);
    base[ire] = h;
    base[(size_t)Qp * K2 + ire] = l;
    split_pair(v.y, h, l);
    base[iim] = h;
    base[(size_t)Qp * K2 + iim] = l;
}

// Xb[leaf][chunk][plane][ncol][2 Qp]: column n of chunk ch is right-hand side
// ch ncol + n; row k < Qp: Re x at slot k of the leaf, k >= Qp: Im x at slot k - Qp
__global__ void k_xnb_prep(int64_t nleaf, int nF, int Qp, int r, int ncol, int nchunk, const int32_t *leafdof,
                           const double2 *xt, __bf16 *Xb)
{
    const int K2 = 2 * Qp;
    const int64_t per = (int64_t)ncol * K2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nleaf * nchunk * per) return;
    const int64_t lc = t / per;
    const int rem = (int)(t % per), n = rem / K2, k = rem % K2;
    const int64_t leaf = lc / nchunk;
    const int ch = (int)(lc % nchunk), col = ch * ncol + n, j = k < Qp ? k : k - Qp;
    double v = 0.0;
    if (j < nF && col < r) {
        const int d = leafdof[(size_t)leaf * nF + j];
        if (d >= 0) {
            const double2 x = xt[(size_t)d * r + col];
            v = k < Qp ? x.x : x.y;
        }
    }
    __bf16 h, l;
    split_pair(v, h, l);
    __bf16 *base = Xb + (size_t)lc * 2 * per;
    base[rem] = h;
    base[per + rem] = l;
}

template <int QP, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_near_bx(int r, int nchunk, int nF, int64_t nwork,
                                                 const int32_t *order, const M2LWork *work, const int32_t *partner,
                                                 const int32_t *aslot, const __bf16 *Ab, const __bf16 *Xb,
                                                 float2 *part)
{
    // QP: slots rounded up to 32.  The right factor of each reduction step (all columns,
    // 32 slots, re and im, both planes) is staged once per workgroup in shared memory,
    // double-buffered: the next step's share is loaded during the current products and
    // stored after them (one barrier per step).  The left factor rows of each wave are
    // read straight from memory (no wave shares them).
    constexpr int NCOL = 16 * NT, Qp = QP, K2 = 2 * QP, KS = QP / 32, MTT = QP / 16, MTW = (MTT + 3) / 4;
    constexpr int LDX = 72;                    // staged column: 32 re + 32 im + padding
    constexpr int XP = 2 * NCOL * 2 * 4;       // 16-byte pieces per step: planes, columns, re/im, 4
    constexpr int XV = (XP + 255) / 256;       // pieces per thread
    __shared__ __bf16 sX[2][2][NCOL][LDX];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // the chunks of one work item share an XCD (consecutive ids go round-robin over 8)
    const int64_t g = blockIdx.x;
    const int64_t wo = (g / (8 * nchunk)) * 8 + g % 8;
    const int ch = (int)((g / 8) % nchunk);
    if (wo >= nwork) return;
    const int64_t wi = order[wo];
    const M2LWork wk = work[wi];
    const size_t aper = (size_t)2 * Qp * K2, xper = (size_t)NCOL * K2;
    auto xsrc = [&](int kp) { return Xb + ((size_t)partner[kp] * nchunk + ch) * 2 * xper; };
    // piece e of step s: plane, column, re/im, quarter (quarters of one 64-byte run adjacent)
    auto x_load = [&](const __bf16 *Xs, int s, int e) -> uint4 {
        const int q = e & 3, h = (e >> 2) & 1, n = (e >> 3) % NCOL, pl = (e >> 3) / NCOL;
        return *reinterpret_cast<const uint4 *>(Xs + pl * xper + (size_t)n * K2 + h * Qp + 32 * s + 8 * q);
    };
    auto x_store = [&](int buf, int e, uint4 v) {
        const int q = e & 3, h = (e >> 2) & 1, n = (e >> 3) % NCOL, pl = (e >> 3) / NCOL;
        *reinterpret_cast<uint4 *>(&sX[buf][pl][n][32 * h + 8 * q]) = v;
    };
    f4 ar[MTW][NT], ai[MTW][NT];
#pragma unroll
    for (int a = 0; a < MTW; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            ar[a][t] = f4{0.f, 0.f, 0.f, 0.f};
            ai[a][t] = f4{0.f, 0.f, 0.f, 0.f};
        }
    {   // first step straight into buffer 0
        const __bf16 *Xs = xsrc(wk.beg);
#pragma unroll
        for (int v = 0; v < XV; ++v) {
            const int e = tid + 256 * v;
            if (XP % 256 == 0 || e < XP) x_store(0, e, x_load(Xs, 0, e));
        }
    }
    __syncthreads();
    int buf = 0;
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const __bf16 *As = Ab + (size_t)aslot[kp] * aper;
        const __bf16 *Xs = xsrc(kp);
        const __bf16 *Xn = xsrc(min(kp + 1, wk.end - 1));   // (the last partner again at the end)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            // the next step's share of the right factor, in flight during the products
            uint4 pc[XV];
#pragma unroll
            for (int v = 0; v < XV; ++v) {
                const int e = tid + 256 * v;
                if (XP % 256 == 0 || e < XP) pc[v] = s + 1 < KS ? x_load(Xs, s + 1, e) : x_load(Xn, 0, e);
            }
            const int k = 32 * s + 8 * (lane >> 4);
            // every row tile of this step loaded before the products (no bounds branch
            // when the tiles divide evenly over the four waves)
            bf8 ba[MTW][2][2];
#pragma unroll
            for (int a = 0; a < MTW; ++a) {
                const int mt = wv * MTW + a;
                if (MTT % 4 != 0 && mt >= MTT) break;   // uniform over the wave
                const __bf16 *arow = As + (size_t)(16 * mt + (lane & 15)) * K2 + k;
#pragma unroll
                for (int pl = 0; pl < 2; ++pl) {
                    ba[a][0][pl] = *reinterpret_cast<const bf8 *>(arow + pl * (size_t)Qp * K2);
                    ba[a][1][pl] = *reinterpret_cast<const bf8 *>(arow + pl * (size_t)Qp * K2 + Qp);
                }
            }
            bf8 xr[NT][2], xi[NT][2];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int pl = 0; pl < 2; ++pl) {
                    const __bf16 *xc = &sX[buf][pl][16 * t + (lane & 15)][8 * (lane >> 4)];
                    xr[t][pl] = *reinterpret_cast<const bf8 *>(xc);
                    xi[t][pl] = *reinterpret_cast<const bf8 *>(xc + 32);
                }
            // Yr += Ar Xr - Ai Xi, Yi += Ai Xr + Ar Xi, each as three split products
            // (hi.hi, hi.lo, lo.hi); the loop over (term, tile, column tile) puts
            // MTW NT independent accumulators between two updates of the same one
#pragma unroll
            for (int term = 0; term < 3; ++term) {
                const int pa = term == 2 ? 1 : 0, px = term == 1 ? 1 : 0;
#pragma unroll
                for (int a = 0; a < MTW; ++a) {
                    const int mt = wv * MTW + a;
                    if (MTT % 4 != 0 && mt >= MTT) break;
                    const bf8 br = ba[a][0][pa], bi = ba[a][1][pa], nb = neg8(bi);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        ar[a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, xr[t][px], ar[a][t], 0, 0, 0);
                        ai[a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bi, xr[t][px], ai[a][t], 0, 0, 0);
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        ar[a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nb, xi[t][px], ar[a][t], 0, 0, 0);
                        ai[a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, xi[t][px], ai[a][t], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < XV; ++v) {
                const int e = tid + 256 * v;
                if (XP % 256 == 0 || e < XP) x_store(buf ^ 1, e, pc[v]);
            }
            __syncthreads();   // next step staged; this step's buffer is free
            buf ^= 1;
        }
    }
    // lane holds D[4 (lane/16) + j][lane % 16] of each tile
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = ch * NCOL + 16 * t + (lane & 15);
        if (col >= r) continue;
#pragma unroll
        for (int a = 0; a < MTW; ++a) {
            const int mt = wv * MTW + a;
            if (MTT % 4 != 0 && mt >= MTT) break;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * mt + 4 * (lane >> 4) + j;
                if (m < nF) part[((size_t)wi * nF + m) * r + col] = make_float2(ar[a][t][j], ai[a][t][j]);
            }
        }
    }
}

// yt[i][c] = sum of the partial results of unknown i (list order), one thread per (i, c)
__global__ void k_nb_gather(int64_t N, int r, const int64_t *ptr, const int32_t *idx, const float2 *part, double2 *yt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * r) return;
    const int64_t i = t / r;
    const int c = (int)(t % r);
    double re = 0.0, im = 0.0;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const float2 v = part[(size_t)idx[k] * r + c];
        re += v.x;
        im += v.y;
    }
    yt[t] = make_double2(re, im);
}

// FP64 blocks Ad[2 b + ori][Qp][2 Qp] ([Re | Im] rows, ori as for Ab)
__global__ void k_nd_store(const double2 *bval, int64_t nblk, int nF, int Qp, double *Ad)
{
    const int K2 = 2 * Qp;
    const int64_t per = (int64_t)Qp * Qp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * nblk * per) return;
    const int64_t po = t / per;
    const int rem = (int)(t % per), i = rem / Qp, j = rem % Qp;
    const int64_t b = po / 2;
    const int ori = (int)(po % 2);
    double2 v = make_double2(0.0, 0.0);
    if (i < nF && j < nF) v = ori == 0 ? bval[((size_t)b * nF + i) * nF + j] : bval[((size_t)b * nF + j) * nF + i];
    double *base = Ad + (size_t)po * Qp * K2;
    base[(size_t)i * K2 + j] = v.x;
    base[(size_t)i * K2 + Qp + j] = v.y;
}

// Xd[leaf][chunk][ncol][2 Qp] FP64: column n of chunk ch is right-hand side ch ncol + n
__global__ void k_xnd_prep(int64_t nleaf, int nF, int Qp, int r, int ncol, int nchunk, const int32_t *leafdof,
                           const double2 *xt, double *Xd)
{
    const int K2 = 2 * Qp;
    const int64_t per = (int64_t)ncol * K2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nleaf * nchunk * per) return;
    const int64_t lc = t / per;
    const int rem = (int)(t % per), n = rem / K2, k = rem % K2;
    const int64_t leaf = lc / nchunk;
    const int ch = (int)(lc % nchunk), col = ch * ncol + n, j = k < Qp ? k : k - Qp;
    double v = 0.0;
    if (j < nF && col < r) {
        const int d = leafdof[(size_t)leaf * nF + j];
        if (d >= 0) {
            const double2 x = xt[(size_t)d * r + col];
            v = k < Qp ? x.x : x.y;
        }
    }
    Xd[(size_t)lc * per + rem] = v;
}

// FP64 real product (16x16x4 FP64 instruction: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register j of lane l holds D[l/16 + 4j][l%16]).  Waves:
// wm = 0 real rows, 1 imaginary rows; wr = row half (MTW row tiles each); wn = column
// group of NT tiles.  Two instructions take eight consecutive reduction indices, lane
// group g the pair 2g, 2g + 1 (one 16-byte load per lane feeds both); the operands of
// the next step are loaded during the products of the current one.
typedef double dx4n __attribute__((ext_vector_type(4)));
template <int MTW, int WN, int NT>
__global__ __launch_bounds__(256 * WN) void k_near_md(int r, int nchunk, int nF, int64_t nwork, const int32_t *order,
                                                      const M2LWork *work, const int32_t *partner,
                                                      const int32_t *aslot, const double *Ad, const double *Xd,
                                                      double2 *part)
{
    constexpr int QP = 32 * MTW, K2 = 2 * QP, NCOL = 16 * WN * NT, KS = K2 / 8;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv / (2 * WN), wr = (wv / WN) % 2, wn = wv % WN;
    const int gi = lane >> 4, li = lane & 15;
    const int64_t g = blockIdx.x;
    const int64_t wo = (g / (8 * nchunk)) * 8 + g % 8;
    const int ch = (int)((g / 8) % nchunk);
    if (wo >= nwork) return;
    const M2LWork wk = work[order[wo]];
    const int64_t wi = order[wo];
    const size_t aper = (size_t)QP * K2, xper = (size_t)NCOL * K2;
    dx4n acc[MTW][NT];
#pragma unroll
    for (int a = 0; a < MTW; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[a][t] = dx4n{0.0, 0.0, 0.0, 0.0};
    const int nstep = (wk.end - wk.beg) * KS;
    double2 av[MTW], bv[NT];
    auto load = [&](int it) {
        const int kp = wk.beg + it / KS, s8 = it % KS;
        const double *Ap = Ad + (size_t)aslot[kp] * aper;
        const double *Xs = Xd + ((size_t)partner[kp] * nchunk + ch) * xper;
        const int kb = 8 * s8 + 2 * gi;
        // real rows [Br, -Bi], imaginary rows [Bi, Br] of the stored [Br | Bi]; kb and
        // 8 s8 lie in the same half (QP is a multiple of 16)
        const bool hi = 8 * s8 >= QP;
        const int ksrc = wm == 0 ? kb : (hi ? kb - QP : kb + QP);
#pragma unroll
        for (int t = 0; t < NT; ++t)
            bv[t] = *reinterpret_cast<const double2 *>(Xs + (size_t)(16 * (wn * NT + t) + li) * K2 + kb);
#pragma unroll
        for (int a = 0; a < MTW; ++a)
            av[a] = *reinterpret_cast<const double2 *>(Ap + (size_t)(16 * (wr * MTW + a) + li) * K2 + ksrc);
        return wm == 0 && hi;
    };
    bool neg = nstep > 0 ? load(0) : false;
    for (int it = 0; it < nstep; ++it) {
        double2 ca[MTW], cb[NT];
#pragma unroll
        for (int a = 0; a < MTW; ++a) ca[a] = neg ? make_double2(-av[a].x, -av[a].y) : av[a];
#pragma unroll
        for (int t = 0; t < NT; ++t) cb[t] = bv[t];
        if (it + 1 < nstep) neg = load(it + 1);
#pragma unroll
        for (int a = 0; a < MTW; ++a)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[a][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[a].x, cb[t].x, acc[a][t], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < MTW; ++a)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[a][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[a].y, cb[t].y, acc[a][t], 0, 0, 0);
    }
    // lane holds D[lane/16 + 4 j][lane % 16] of each tile: slot m, column n
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = ch * NCOL + 16 * (wn * NT + t) + li;
        if (col >= r) continue;
#pragma unroll
        for (int a = 0; a < MTW; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * (wr * MTW + a) + gi + 4 * j;
                if (m < nF) reinterpret_cast<double *>(part + ((size_t)wi * nF + m) * r + col)[wm] = acc[a][t][j];
            }
    }
}

__global__ void k_nd_gather(int64_t N, int r, const int64_t *ptr, const int32_t *idx, const double2 *part, double2 *yt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * r) return;
    const int64_t i = t / r;
    const int c = (int)(t % r);
    double re = 0.0, im = 0.0;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const double2 v = part[(size_t)idx[k] * r + c];
        re += v.x;
        im += v.y;
    }
    yt[t] = make_double2(re, im);
}

int near_qp(int nF) { return 32 * ((nF + 31) / 32); }

}  // namespace

void plan_near_bf16(ige_op op, const std::vector<int32_t> &pair, const std::vector<int32_t> &leafdof, int nF)
{
    const int64_t nblk = (int64_t)pair.size() / 2;
    const int64_t nleaf = nF > 0 ? (int64_t)leafdof.size() / nF : 0;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lst(nleaf);   // per target: (source leaf, block slot)
    for (int64_t b = 0; b < nblk; ++b) {
        const int lt = pair[2 * b], ls = pair[2 * b + 1];
        lst[lt].push_back({ls, (int32_t)(2 * b)});
        if (lt != ls) lst[ls].push_back({lt, (int32_t)(2 * b + 1)});
    }
    std::vector<M2LWork> work;
    std::vector<int32_t> partner, aslot;
    for (int64_t t = 0; t < nleaf; ++t) {
        std::sort(lst[t].begin(), lst[t].end());
        const int beg = (int)partner.size();
        for (const auto &e : lst[t]) {
            partner.push_back(e.first);
            aslot.push_back(e.second);
        }
        for (int b = beg; b < (int)partner.size(); b += kNearPartners)
            work.push_back({(int32_t)t, b, std::min((int)partner.size(), b + kNearPartners)});
    }
    std::vector<int32_t> order(work.size());
    for (size_t w = 0; w < order.size(); ++w) order[w] = (int32_t)w;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return work[a].end - work[a].beg > work[b].end - work[b].beg;
    });
    // per unknown: the partial-result rows (work item, slot) that hold it, in order
    const int64_t N = op->D.N;
    std::vector<int64_t> ptr(N + 1, 0);
    for (const auto &w : work)
        for (int j = 0; j < nF; ++j) {
            const int d = leafdof[(size_t)w.tgt * nF + j];
            if (d >= 0) ptr[d + 1]++;
        }
    for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
    std::vector<int32_t> idx(ptr[N]);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t w = 0; w < work.size(); ++w)
        for (int j = 0; j < nF; ++j) {
            const int d = leafdof[(size_t)work[w].tgt * nF + j];
            if (d >= 0) idx[fill[d]++] = (int32_t)(w * nF + j);
        }
    hipStream_t s = op->ctx->stream;
    op->nb_nwork = (int64_t)work.size();
    op->d_nbwork.upload(work, s);
    op->d_nbpartner.upload(partner, s);
    op->d_nbslot.upload(aslot, s);
    op->d_nborder.upload(order, s);
    op->d_nbred_ptr.upload(ptr, s);
    op->d_nbred_idx.upload(idx, s);
}

// the split-BF16 blocks, made on first use on the stream of the product that reads them
void ensure_near_bf16(ige_op op, hipStream_t s)
{
    if (op->d_nb3.p || op->view.nblk == 0) return;
    const DevOp &o = op->view;
    const int Qp = near_qp(o.nF);
    op->d_nb3.alloc((size_t)2 * o.nblk * 2 * Qp * 2 * Qp);
    const int64_t n = 2 * o.nblk * (int64_t)Qp * Qp;
    hipLaunchKernelGGL(k_nb_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, o.bval, o.nblk, o.nF, Qp,
                       op->d_nb3.p);
    IGE_HIP(hipGetLastError());
}

int near_bf16_ok(int nF) { return near_qp(nF) / 16 <= 4 * 4; }

namespace {
template <int QP, int NT>
void launch_bx(ige_op op, int r, int nchunk, hipStream_t s)
{
    const DevOp &o = op->view;
    const int64_t nw = op->nb_nwork;
    if (nw == 0) return;
    const dim3 grid((unsigned)(((nw + 7) / 8) * 8 * nchunk)), blk(256);
    hipLaunchKernelGGL((k_near_bx<QP, NT>), grid, blk, 0, s, r, nchunk, o.nF, nw, op->d_nborder.p, op->d_nbwork.p,
                       op->d_nbpartner.p, op->d_nbslot.p, op->d_nb3.p, op->d_xnb.p, op->d_nbpart.p);
    IGE_HIP(hipGetLastError());
}

template <int QP>
void launch_bx_nt(ige_op op, int r, int NT, int nchunk, hipStream_t s)
{
    switch (NT) {
        case 1: launch_bx<QP, 1>(op, r, nchunk, s); break;
        case 2: launch_bx<QP, 2>(op, r, nchunk, s); break;
        default: launch_bx<QP, 4>(op, r, nchunk, s); break;
    }
}
}  // namespace

void near_bf16(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s)
{
    const DevOp &o = op->view;
    IGE_REQUIRE(near_bf16_ok(o.nF), "near-field blocks too large for the split-BF16 product");
    ensure_near_bf16(op, s);
    const int Qp = near_qp(o.nF);
    int NT = tune_get(op, kTuneNearBxNt, r, 0, r > 32 ? 4 : (r > 16 ? 2 : 1));
    if (NT != 1 && NT != 2) NT = 4;
    if (NT == 4 && (Qp == 160 || Qp > 192)) NT = 2;   // four column tiles would spill registers there
    const int ncol = 16 * NT, nchunk = (r + ncol - 1) / ncol;
    const int64_t nleaf = (int64_t)o.P * o.SL * o.SL;
    const size_t xn = (size_t)nleaf * nchunk * 2 * ncol * 2 * Qp;
    if (op->d_xnb.n < xn) op->d_xnb.alloc(xn);
    const size_t pn = (size_t)op->nb_nwork * o.nF * r;
    if (op->d_nbpart.n < pn) op->d_nbpart.alloc(pn);
    const int64_t nx = (int64_t)nleaf * nchunk * ncol * 2 * Qp;
    hipLaunchKernelGGL(k_xnb_prep, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, nleaf, o.nF, Qp, r, ncol,
                       nchunk, o.leafdof, xt, op->d_xnb.p);
    IGE_HIP(hipGetLastError());
    switch (Qp) {
        case 32: launch_bx_nt<32>(op, r, NT, nchunk, s); break;
        case 64: launch_bx_nt<64>(op, r, NT, nchunk, s); break;
        case 96: launch_bx_nt<96>(op, r, NT, nchunk, s); break;
        case 128: launch_bx_nt<128>(op, r, NT, nchunk, s); break;
        case 160: launch_bx_nt<160>(op, r, NT, nchunk, s); break;
        case 192: launch_bx_nt<192>(op, r, NT, nchunk, s); break;
        case 224: launch_bx_nt<224>(op, r, NT, nchunk, s); break;
        default: launch_bx_nt<256>(op, r, NT, nchunk, s); break;
    }
    const int64_t tot = (int64_t)o.N * r;
    hipLaunchKernelGGL(k_nb_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (int64_t)o.N, r,
                       op->d_nbred_ptr.p, op->d_nbred_idx.p, op->d_nbpart.p, yt);
    IGE_HIP(hipGetLastError());
}


// FP64 matrix-core near field for many columns: blocks made on first use when they
// leave 8 GiB of device memory free.  Ordered pairs read each block twice (as itself
// and as its transpose) where the unordered-block kernel reads it once for both
// products, so they pay only once the products dominate: from 56 columns (measured
// at 8, 16, 32 and 64 columns with chunks of 16, 32 and 64)
bool near_f64mx_ok(ige_op op, int r)
{
    const DevOp &o = op->view;
    if (r < 56 || o.nblk == 0 || op->near_md_off || near_qp(o.nF) > 256) return false;
    if (op->nd_fit < 0) {   // decided once, at the first eligible apply (never under capture)
        const int Qp = near_qp(o.nF);
        const size_t need = (size_t)2 * o.nblk * Qp * 2 * Qp * sizeof(double);
        size_t fr = 0, tot = 0;
        IGE_HIP(hipMemGetInfo(&fr, &tot));
        op->nd_fit = op->d_nd.p || need + ((size_t)8 << 30) < fr ? 1 : 0;
    }
    return op->nd_fit == 1;
}

namespace {
// 64 columns per workgroup as two column waves of two tiles (one column wave of four
// tiles, or four of one, measured no faster)
template <int MTW>
void launch_nd(ige_op op, int r, int nchunk, hipStream_t s)
{
    constexpr int WN = 2, NT = 2;
    const DevOp &o = op->view;
    const int64_t nw = op->nb_nwork;
    if (nw == 0) return;
    const dim3 grid((unsigned)(((nw + 7) / 8) * 8 * nchunk)), blk(256 * WN);
    hipLaunchKernelGGL((k_near_md<MTW, WN, NT>), grid, blk, 0, s, r, nchunk, o.nF, nw, op->d_nborder.p,
                       op->d_nbwork.p, op->d_nbpartner.p, op->d_nbslot.p, op->d_nd.p, op->d_xnd.p, op->d_ndpart.p);
    IGE_HIP(hipGetLastError());
}
}  // namespace

void near_f64mx(ige_op op, int r, const double2 *xt, double2 *yt, hipStream_t s)
{
    const DevOp &o = op->view;
    const int Qp = near_qp(o.nF);
    if (!op->d_nd.p) {
        op->d_nd.alloc((size_t)2 * o.nblk * Qp * 2 * Qp);
        const int64_t n = 2 * o.nblk * (int64_t)Qp * Qp;
        hipLaunchKernelGGL(k_nd_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, o.bval, o.nblk, o.nF, Qp,
                           op->d_nd.p);
        IGE_HIP(hipGetLastError());
    }
    constexpr int ncol = 64;   // columns per workgroup
    const int nchunk = (r + ncol - 1) / ncol;
    const int64_t nleaf = (int64_t)o.P * o.SL * o.SL;
    const size_t xn = (size_t)nleaf * nchunk * ncol * 2 * Qp;
    if (op->d_xnd.n < xn) op->d_xnd.alloc(xn);
    const size_t pn = (size_t)op->nb_nwork * o.nF * r;
    if (op->d_ndpart.n < pn) op->d_ndpart.alloc(pn);
    hipLaunchKernelGGL(k_xnd_prep, dim3((unsigned)(((int64_t)xn + 255) / 256)), dim3(256), 0, s, nleaf, o.nF, Qp, r,
                       ncol, nchunk, o.leafdof, xt, op->d_xnd.p);
    IGE_HIP(hipGetLastError());
    switch (Qp / 32) {
        case 1: launch_nd<1>(op, r, nchunk, s); break;
        case 2: launch_nd<2>(op, r, nchunk, s); break;
        case 3: launch_nd<3>(op, r, nchunk, s); break;
        case 4: launch_nd<4>(op, r, nchunk, s); break;
        case 5: launch_nd<5>(op, r, nchunk, s); break;
        case 6: launch_nd<6>(op, r, nchunk, s); break;
        case 7: launch_nd<7>(op, r, nchunk, s); break;
        default: launch_nd<8>(op, r, nchunk, s); break;
    }
    const int64_t tot = (int64_t)o.N * r;
    hipLaunchKernelGGL(k_nd_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (int64_t)o.N, r,
                       op->d_nbred_ptr.p, op->d_nbred_idx.p, op->d_ndpart.p, yt);
    IGE_HIP(hipGetLastError());
}

}  // namespace ige
