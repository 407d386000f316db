// Coupling stage (M2L) on the matrix cores, for many right-hand sides: BF16 and split
// BF16 (below), and FP64 (the last kernels of this file).
//
// The kernel matrices G of the admissible pairs (the dense coupling blocks of the
// interpolation-based FMM, Sec. 4) are stored once in BF16, in both orientations
// (G_ts and G_st = G_ts^T, rows [Re | Im]), so that the operand of every ordered pair
// t <- s has its reduction index contiguous.  A complex product U_t = G_ts V_s over
// all right-hand sides is one real product with stacked real and imaginary parts,
//   [Re U; Im U] (2Qp x n) = [[Gr, -Gi], [Gi, Gr]] (2Qp x 2Qp) . [Re V; Im V] (2Qp x n),
// whose left factor is read from the stored [Gr | Gi] rows (halves swapped for the
// imaginary rows, sign flipped on the Gi half of the real rows), so the streamed
// right factor holds each complex entry once.  The product runs on the 16x16x32
// BF16 instruction with FP32 accumulation (lane l supplies A[l%16][8(l/16)+i] and
// B[8(l/16)+i][l%16]; accumulator register j of lane l holds D[4(l/16)+j][l%16]).
// With split = 3 both factors are stored as a BF16 pair (x = xh + xl) and the
// product is xh.yh + xh.yl + xl.yh (about 2^-16 relative).
//
// Work: one workgroup per (work item = target cluster and up to 32 partners, column
// chunk of up to 64 right-hand sides), all columns of the chunk at once so that each
// block G is read once per chunk: G is staged in shared memory (the next partner's
// block prefetched into registers during the current product), the right factor is
// streamed from memory into registers one reduction step ahead.  Wave wm = 0 forms
// the real rows, wm = 1 the imaginary rows; wn splits the columns.  Partial couplings
// per work item (FP32) are summed by the fixed-order per-cluster reduction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.hpp"
#include "op.hpp"

#ifndef IGE_GPAD
#define IGE_GPAD 8   // padding (BF16 elements) of a staged block row in shared memory
#endif

namespace ige {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline void split_bf16(double x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)(float)x;
    lo = (__bf16)(float)(x - (double)(float)hi);
}

// G in BF16: Gb[(2 pair + orientation) * planes + plane][Qp][2Qp] (planes = 2 for the
// split form: high and low part, else 1); orientation 0 =
// G_ts (rows: nodes of t), 1 = G_st; columns [Re | Im], zero padded
// (Qr nodes per cluster, of the stride o.Q of the cluster arrays: the degree of the
// pairs' level)
__global__ void k_gb_store(DevOp o, int64_t nfp, const int32_t *fpair, int Qr, int Qp, int split, __bf16 *Gb)
{
    const int Qs = o.Q, Q = Qr, K2 = 2 * Qp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)Qp * Qp;
    if (t >= nfp * 2 * per) return;
    const int64_t po = t / per;   // 2 pair + orientation
    const int r = (int)(t % per), m = r / Qp, mc = r % Qp;
    const int64_t pr = po / 2;
    const int ori = (int)(po % 2);
    const int ga = fpair[2 * pr + ori], gb = fpair[2 * pr + 1 - ori];
    double2 g = make_double2(0.0, 0.0);
    if (m < Q && mc < Q) {
        const double *Xa = o.nodeX + (size_t)ga * 3 * Qs, *Xb = o.nodeX + (size_t)gb * 3 * Qs;
        const double d0 = Xa[m] - Xb[mc], d1 = Xa[Qs + m] - Xb[Qs + mc], d2 = Xa[2 * Qs + m] - Xb[2 * Qs + mc];
        g = dm::helmholtz_r2_tab(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2)), o.sctab);
    }
    __bf16 *base = Gb + (size_t)po * (split == 3 ? 2 : 1) * Qp * K2;
    const size_t i_re = (size_t)m * K2 + mc, i_im = i_re + Qp;
    if (split == 1) {
        base[i_re] = (__bf16)(float)g.x;
        base[i_im] = (__bf16)(float)g.y;
    } else {
        __bf16 h, l;
        split_bf16(g.x, h, l);
        base[i_re] = h;
        base[(size_t)Qp * K2 + i_re] = l;
        split_bf16(g.y, h, l);
        base[i_im] = h;
        base[(size_t)Qp * K2 + i_im] = l;
    }
}

// Source fields [NC][4][Q][r] -> right factor Vb[cluster][chunk][plane][ncol][2Qp]
// (planes as for G): column n = f rc + j (field f, right-hand side ch rc + j),
// row k < Qp: Re V[k], k >= Qp: Im V[k - Qp]; zero padded
// (clusters cl0 .. cl0 + NC - 1 with Qr nodes each, at Vb[cluster - cl0])
__global__ void k_vb_prep(DevOp o, int NC, int cl0, int Qr, int r, int rc, int nchunk, int ncol, int Qp, int split,
                          const double2 *src, __bf16 *Vb)
{
    const int Qs = o.Q, Q = Qr, K2 = 2 * Qp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)ncol * K2;
    if (t >= (int64_t)NC * nchunk * per) return;
    const int64_t cc = t / per;   // cluster * nchunk + chunk
    const int rem = (int)(t % per), n = rem / K2, k = rem % K2;
    const int gc = (int)(cc / nchunk), ch = (int)(cc % nchunk);
    const int f = n / rc, j = n % rc, col = ch * rc + j;
    const int mm = k < Qp ? k : k - Qp;
    double v = 0.0;
    if (mm < Q && col < r && f < 4) {
        const double2 s = src[(((size_t)(cl0 + gc) * 4 + f) * Qs + mm) * r + col];
        v = k < Qp ? s.x : s.y;
    }
    __bf16 *base = Vb + (size_t)cc * (split == 3 ? 2 : 1) * per;
    if (split == 1) {
        base[rem] = (__bf16)(float)v;
    } else {
        __bf16 hi, lo;
        split_bf16(v, hi, lo);
        base[rem] = hi;
        base[per + rem] = lo;
    }
}

// The same conversion through shared memory: a workgroup takes 32 nodes of one field
// of one cluster and one column chunk, reads them along the columns (coalesced, the
// layout of src) and writes each column's 32-node runs of Re and Im (contiguous in Vb).
constexpr int kVbRows = 32;
__global__ __launch_bounds__(256) void k_vb_prep_t(DevOp o, int cl0, int Qr, int r, int rc, int nchunk, int ncol,
                                                   int Qp, int split, const double2 *src, __bf16 *Vb)
{
    __shared__ double2 tile[kVbRows][65];   // [node][column in chunk], rc <= 64
    const int Qs = o.Q, Q = Qr, K2 = 2 * Qp, nrb = Qp / kVbRows;
    int b = blockIdx.x;
    const int rb = b % nrb;
    b /= nrb;
    const int f = b % 4;
    b /= 4;
    const int ch = b % nchunk, gc = b / nchunk;
    const int m0 = rb * kVbRows;
    for (int i = threadIdx.x; i < kVbRows * rc; i += blockDim.x) {
        const int mm = i / rc, j = i % rc, col = ch * rc + j, m = m0 + mm;
        tile[mm][j] = (m < Q && col < r) ? src[(((size_t)(cl0 + gc) * 4 + f) * Qs + m) * r + col] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int64_t per = (int64_t)ncol * K2;
    __bf16 *base = Vb + ((size_t)gc * nchunk + ch) * (split == 3 ? 2 : 1) * per;
    for (int i = threadIdx.x; i < rc * 2 * kVbRows; i += blockDim.x) {
        const int j = i / (2 * kVbRows), h = (i / kVbRows) & 1, mm = i % kVbRows;
        const double2 t = tile[mm][j];
        const double v = h ? t.y : t.x;
        const size_t at = (size_t)(f * rc + j) * K2 + h * Qp + m0 + mm;
        if (split == 1) {
            base[at] = (__bf16)(float)v;
        } else {
            __bf16 hi, lo;
            split_bf16(v, hi, lo);
            base[at] = hi;
            base[per + at] = lo;
        }
    }
}

__device__ inline bf8 neg_bf8(bf8 x)
{
    uint4 u = __builtin_bit_cast(uint4, x);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(bf8, u);
}

// MT = Qp / 16 row tiles per wave, WN column waves of NT 16-column tiles each:
// 2 WN waves, ncol = 16 WN NT columns per chunk
template <int SPLIT, int MT, int WN, int NT>
__global__ __launch_bounds__(128 * WN) void k_m2l_mx(DevOp o, int r, int rc, int nchunk, int64_t nwork, int Qr, int cl0,
                                                     const int32_t *order, const M2LWork *work,
                                                     const int32_t *partner, const int32_t *gslot, const __bf16 *Gb,
                                                     const __bf16 *Vb, float2 *part)
{
    constexpr int PL = SPLIT == 3 ? 2 : 1;   // BF16 planes per factor
    constexpr int QP = 16 * MT, K2 = 2 * QP, KS = K2 / 32, LD = K2 + IGE_GPAD;
    constexpr int NTH = 128 * WN, NCOL = 16 * WN * NT;
    constexpr int GCH = PL * QP * K2 / 8;           // 16-byte pieces of one block
    constexpr int GV = (GCH + NTH - 1) / NTH;       // pieces per thread
    constexpr bool PREF = GV <= 16;                 // next block prefetched into registers
    extern __shared__ __bf16 sG[];                  // [PL][QP][LD]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv / WN, wn = wv % WN;
    const int Q = o.Q;   // stride of the partial couplings; Qr rows of them written
    // the chunks of one work item share an XCD (consecutive ids go round-robin over 8)
    const int64_t g = blockIdx.x;
    const int64_t wo = (g / (8 * nchunk)) * 8 + g % 8;
    const int ch = (int)((g / 8) % nchunk);
    if (wo >= nwork) return;
    const int64_t wi = order[wo];
    if (wi < 0) return;   // padding slot of a launch order
    const M2LWork wk = work[wi];
    if (wk.beg >= wk.end) return;
    const size_t gper = (size_t)PL * QP * K2, vper = (size_t)NCOL * K2;

    auto g_piece = [&](const __bf16 *Gp, int e) -> uint4 {
        return *reinterpret_cast<const uint4 *>(Gp + (size_t)8 * e);
    };
    auto s_piece = [&](int e, uint4 v) {
        const int pl = e / (QP * K2 / 8), rr = e % (QP * K2 / 8), row = rr / (K2 / 8), k8 = rr % (K2 / 8);
        *reinterpret_cast<uint4 *>(sG + ((size_t)pl * QP + row) * LD + 8 * k8) = v;
    };
    auto b_load = [&](bf8 (&b)[NT][PL], int kp, int s) {
        const __bf16 *Vs = Vb + ((size_t)(partner[kp] - cl0) * nchunk + ch) * PL * vper;
        const int kk = 32 * s + 8 * (lane >> 4);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = 16 * (wn * NT + t) + (lane & 15);
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
                b[t][pl] = *reinterpret_cast<const bf8 *>(Vs + (size_t)pl * vper + (size_t)n * K2 + kk);
        }
    };

    f4 acc[MT][NT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[a][t] = f4{0.f, 0.f, 0.f, 0.f};

    // loads stay branch-free so that the waits before the products count only the
    // loads they need: piece indices are checked only when the pieces do not divide
    // evenly, and the prefetch after the last partner re-reads the last block
    constexpr bool GEVEN = GCH % NTH == 0;
    uint4 gpre[PREF ? GV : 1];
    if (PREF) {
        const __bf16 *Gp = Gb + (size_t)gslot[wk.beg] * gper;
#pragma unroll
        for (int v = 0; v < GV; ++v) {
            const int e = tid + NTH * v;
            if (GEVEN || e < GCH) gpre[v] = g_piece(Gp, e);
        }
    }
    bf8 bcur[NT][PL], bnxt[NT][PL];
    b_load(bcur, wk.beg, 0);
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        __syncthreads();   // every wave is done with the previous block
        if (PREF) {
#pragma unroll
            for (int v = 0; v < GV; ++v) {
                const int e = tid + NTH * v;
                if (GEVEN || e < GCH) s_piece(e, gpre[v]);
            }
        } else {
            const __bf16 *Gp = Gb + (size_t)gslot[kp] * gper;
            for (int e = tid; e < GCH; e += NTH) s_piece(e, g_piece(Gp, e));
        }
        __syncthreads();
        const int kq = min(kp + 1, wk.end - 1);   // next partner (the last one again at the end)
        if (PREF) {
            const __bf16 *Gp = Gb + (size_t)gslot[kq] * gper;
#pragma unroll
            for (int v = 0; v < GV; ++v) {
                const int e = tid + NTH * v;
                if (GEVEN || e < GCH) gpre[v] = g_piece(Gp, e);
            }
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s + 1 < KS) b_load(bnxt, kp, s + 1);
            else b_load(bnxt, kq, 0);
            // left factor: real rows [Gr, -Gi], imaginary rows [Gi, Gr] of the stored [Gr | Gi]
            const bool hi_half = 32 * s >= QP;
            const int kk = 32 * s + 8 * (lane >> 4);
            const int ksrc = wm == 0 ? kk : (hi_half ? kk - QP : kk + QP);
            const bool neg = wm == 0 && hi_half;
            // row tiles in pairs; the three split products go over the pair's 2 NT
            // accumulators in turn, so consecutive instructions never share an accumulator
#pragma unroll
            for (int a0 = 0; a0 < MT; a0 += 2) {
                constexpr int NA = 2;
                bf8 ah[NA], al[NA];
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    if (a0 + u >= MT) break;
                    const __bf16 *row = sG + (size_t)(16 * (a0 + u) + (lane & 15)) * LD + ksrc;
                    ah[u] = *reinterpret_cast<const bf8 *>(row);
                    if (SPLIT == 3) al[u] = *reinterpret_cast<const bf8 *>(row + (size_t)QP * LD);
                    if (neg) {
                        ah[u] = neg_bf8(ah[u]);
                        if (SPLIT == 3) al[u] = neg_bf8(al[u]);
                    }
                }
#pragma unroll
                for (int term = 0; term < (SPLIT == 3 ? 3 : 1); ++term)
#pragma unroll
                    for (int u = 0; u < NA; ++u) {
                        if (a0 + u >= MT) break;
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            const bf8 &A = term == 2 ? al[u] : ah[u];
                            const bf8 &Bv = term == 1 ? bcur[t][PL - 1] : bcur[t][0];
                            acc[a0 + u][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv, acc[a0 + u][t], 0, 0, 0);
                        }
                    }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl) bcur[t][pl] = bnxt[t][pl];
        }
    }
    // lane holds D[4 (lane/16) + j][lane % 16] of each tile: node m, column n = f rc + jc;
    // wave half wm gives the real (0) or imaginary (1) part
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = 16 * (wn * NT + t) + (lane & 15), f = n / rc, jc = n % rc;
        const int col = ch * rc + jc;
        if (f >= 4 || col >= r) continue;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * a + 4 * (lane >> 4) + j;
                if (m < Qr) {
                    float *dst = reinterpret_cast<float *>(part + (((size_t)wi * 4 + f) * Q + m) * r + col);
                    dst[wm] = acc[a][t][j];
                }
            }
    }
}


// The same product with the block staged in two shared-memory buffers: while the
// waves multiply with block kp from one buffer, each reduction step loads a share of
// block kp + 1 into registers and stores it into the other buffer after its products
// (one barrier per partner, a few registers for the pieces in flight instead of the
// whole next block), which leaves room for wider column chunks.
template <int SPLIT, int MT, int WN, int NT>
__global__ __launch_bounds__(128 * WN) void k_m2l_mxd(DevOp o, int r, int rc, int nchunk, int64_t nwork, int Qr, int cl0,
                                                      const int32_t *order, const M2LWork *work,
                                                      const int32_t *partner, const int32_t *gslot, const __bf16 *Gb,
                                                      const __bf16 *Vb, float2 *part)
{
    constexpr int PL = SPLIT == 3 ? 2 : 1;
    constexpr int QP = 16 * MT, K2 = 2 * QP, KS = K2 / 32, LD = K2 + IGE_GPAD;
    constexpr int NTH = 128 * WN, NCOL = 16 * WN * NT;
    constexpr int GCH = PL * QP * K2 / 8;           // 16-byte pieces of one block
    constexpr int GV = (GCH + NTH - 1) / NTH;       // pieces per thread
    constexpr int PPS = (GV + KS - 1) / KS;         // pieces per thread per reduction step
    constexpr size_t BUF = (size_t)PL * QP * LD;    // one staging buffer
    extern __shared__ __bf16 sG[];                  // [2][PL][QP][LD]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv / WN, wn = wv % WN;
    const int Q = o.Q;   // stride of the partial couplings; Qr rows of them written
    const int64_t g = blockIdx.x;
    const int64_t wo = (g / (8 * nchunk)) * 8 + g % 8;
    const int ch = (int)((g / 8) % nchunk);
    if (wo >= nwork) return;
    const int64_t wi = order[wo];
    if (wi < 0) return;   // padding slot of a launch order
    const M2LWork wk = work[wi];
    if (wk.beg >= wk.end) return;
    const size_t gper = (size_t)PL * QP * K2, vper = (size_t)NCOL * K2;

    auto s_piece = [&](__bf16 *buf, int e, uint4 v) {
        const int pl = e / (QP * K2 / 8), rr = e % (QP * K2 / 8), row = rr / (K2 / 8), k8 = rr % (K2 / 8);
        *reinterpret_cast<uint4 *>(buf + ((size_t)pl * QP + row) * LD + 8 * k8) = v;
    };
    auto b_load = [&](bf8 (&b)[NT][PL], int kp, int s) {
        const __bf16 *Vs = Vb + ((size_t)(partner[kp] - cl0) * nchunk + ch) * PL * vper;
        const int kk = 32 * s + 8 * (lane >> 4);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = 16 * (wn * NT + t) + (lane & 15);
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
                b[t][pl] = *reinterpret_cast<const bf8 *>(Vs + (size_t)pl * vper + (size_t)n * K2 + kk);
        }
    };

    f4 acc[MT][NT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[a][t] = f4{0.f, 0.f, 0.f, 0.f};

    {   // first block straight into buffer 0
        const __bf16 *Gp = Gb + (size_t)gslot[wk.beg] * gper;
        for (int e = tid; e < GCH; e += NTH) s_piece(sG, e, *reinterpret_cast<const uint4 *>(Gp + (size_t)8 * e));
    }
    bf8 bcur[NT][PL], bnxt[NT][PL];
    b_load(bcur, wk.beg, 0);
    __syncthreads();
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const __bf16 *cur = sG + (size_t)((kp - wk.beg) & 1) * BUF;
        __bf16 *nxt = sG + (size_t)(((kp - wk.beg) & 1) ^ 1) * BUF;
        // next partner (the last one again at the end: branch-free loads, see above)
        const int kq = min(kp + 1, wk.end - 1);
        const __bf16 *Gn = Gb + (size_t)gslot[kq] * gper;
        constexpr bool GEVEN = GCH % NTH == 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            // this step's share of the next block, in flight during the products
            uint4 pc[PPS];
#pragma unroll
            for (int v = 0; v < PPS; ++v) {
                const int e = tid + NTH * (s * PPS + v);
                if (s * PPS + v < GV && (GEVEN || e < GCH)) pc[v] = *reinterpret_cast<const uint4 *>(Gn + (size_t)8 * e);
            }
            if (s + 1 < KS) b_load(bnxt, kp, s + 1);
            else b_load(bnxt, kq, 0);
            const bool hi_half = 32 * s >= QP;
            const int kk = 32 * s + 8 * (lane >> 4);
            const int ksrc = wm == 0 ? kk : (hi_half ? kk - QP : kk + QP);
            const bool neg = wm == 0 && hi_half;
            // row tiles in pairs; the three split products go over the pair's 2 NT
            // accumulators in turn, so consecutive instructions never share an accumulator
#pragma unroll
            for (int a0 = 0; a0 < MT; a0 += 2) {
                constexpr int NA = 2;
                bf8 ah[NA], al[NA];
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    if (a0 + u >= MT) break;
                    const __bf16 *row = cur + (size_t)(16 * (a0 + u) + (lane & 15)) * LD + ksrc;
                    ah[u] = *reinterpret_cast<const bf8 *>(row);
                    if (SPLIT == 3) al[u] = *reinterpret_cast<const bf8 *>(row + (size_t)QP * LD);
                    if (neg) {
                        ah[u] = neg_bf8(ah[u]);
                        if (SPLIT == 3) al[u] = neg_bf8(al[u]);
                    }
                }
#pragma unroll
                for (int term = 0; term < (SPLIT == 3 ? 3 : 1); ++term)
#pragma unroll
                    for (int u = 0; u < NA; ++u) {
                        if (a0 + u >= MT) break;
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            const bf8 &A = term == 2 ? al[u] : ah[u];
                            const bf8 &Bv = term == 1 ? bcur[t][PL - 1] : bcur[t][0];
                            acc[a0 + u][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv, acc[a0 + u][t], 0, 0, 0);
                        }
                    }
            }
#pragma unroll
            for (int v = 0; v < PPS; ++v) {
                const int e = tid + NTH * (s * PPS + v);
                if (s * PPS + v < GV && (GEVEN || e < GCH)) s_piece(nxt, e, pc[v]);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl) bcur[t][pl] = bnxt[t][pl];
        }
        __syncthreads();   // the next block is complete and the current buffer is free
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = 16 * (wn * NT + t) + (lane & 15), f = n / rc, jc = n % rc;
        const int col = ch * rc + jc;
        if (f >= 4 || col >= r) continue;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * a + 4 * (lane >> 4) + j;
                if (m < Qr) {
                    float *dst = reinterpret_cast<float *>(part + (((size_t)wi * 4 + f) * Q + m) * r + col);
                    dst[wm] = acc[a][t][j];
                }
            }
    }
}


// ---------------------------------------------------------------------------
// The same coupling in FP64 on the FP64 matrix cores (16x16x4: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator register j of lane l holds
// D[l/16 + 4j][l%16]), for many right-hand sides of the FP64 operator.  The blocks
// are stored once in FP64 ([Gr | Gi] rows, both orientations); two instructions take
// eight consecutive reduction indices, lane group g the pair 2g, 2g + 1, so that one
// 16-byte load per lane feeds both.  Left factor rows straight from memory (the four
// column waves of a half read the same rows, served by the caches).
// ---------------------------------------------------------------------------
typedef double dx4m __attribute__((ext_vector_type(4)));

// (Qr nodes per cluster, of the stride o.Q of the cluster arrays, as k_gb_store)
__global__ void k_gd_store(DevOp o, int64_t nfp, const int32_t *fpair, int Qr, int Qp, double *Gd)
{
    const int Qs = o.Q, Q = Qr, K2 = 2 * Qp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)Qp * Qp;
    if (t >= nfp * 2 * per) return;
    const int64_t po = t / per;
    const int rr = (int)(t % per), m = rr / Qp, mc = rr % Qp;
    const int64_t pr = po / 2;
    const int ori = (int)(po % 2);
    const int ga = fpair[2 * pr + ori], gb = fpair[2 * pr + 1 - ori];
    double2 g = make_double2(0.0, 0.0);
    if (m < Q && mc < Q) {
        const double *Xa = o.nodeX + (size_t)ga * 3 * Qs, *Xb = o.nodeX + (size_t)gb * 3 * Qs;
        const double d0 = Xa[m] - Xb[mc], d1 = Xa[Qs + m] - Xb[Qs + mc], d2 = Xa[2 * Qs + m] - Xb[2 * Qs + mc];
        g = dm::helmholtz_r2_tab(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2)), o.sctab);
    }
    double *base = Gd + (size_t)po * Qp * K2;
    base[(size_t)m * K2 + mc] = g.x;
    base[(size_t)m * K2 + Qp + mc] = g.y;
}

// source fields [NC][4][Q][r] -> Vd[cluster][chunk][ncol][2Qp] (FP64), through shared memory
__global__ __launch_bounds__(256) void k_vd_prep_t(DevOp o, int cl0, int Qr, int r, int rc, int nchunk, int ncol,
                                                   int Qp, const double2 *src, double *Vd)
{
    __shared__ double2 tile[kVbRows][65];
    const int Qs = o.Q, Q = Qr, K2 = 2 * Qp, nrb = Qp / kVbRows;
    int b = blockIdx.x;
    const int rb = b % nrb;
    b /= nrb;
    const int f = b % 4;
    b /= 4;
    const int ch = b % nchunk, gc = b / nchunk;
    const int m0 = rb * kVbRows;
    for (int i = threadIdx.x; i < kVbRows * rc; i += blockDim.x) {
        const int mm = i / rc, j = i % rc, col = ch * rc + j, m = m0 + mm;
        tile[mm][j] = (m < Q && col < r) ? src[(((size_t)(cl0 + gc) * 4 + f) * Qs + m) * r + col] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double *base = Vd + ((size_t)gc * nchunk + ch) * (size_t)ncol * K2;
    for (int i = threadIdx.x; i < rc * 2 * kVbRows; i += blockDim.x) {
        const int j = i / (2 * kVbRows), h = (i / kVbRows) & 1, mm = i % kVbRows;
        const double2 t = tile[mm][j];
        base[(size_t)(f * rc + j) * K2 + h * Qp + m0 + mm] = h ? t.y : t.x;
    }
}

template <int MT, int WN, int NT>
__global__ __launch_bounds__(128 * WN) void k_m2l_md(DevOp o, int r, int rc, int nchunk, int64_t nwork, int Qr, int cl0,
                                                     const int32_t *order, const M2LWork *work,
                                                     const int32_t *partner, const int32_t *gslot, const double *Gd,
                                                     const double *Vd, double2 *part)
{
    constexpr int QP = 16 * MT, K2 = 2 * QP, NCOL = 16 * WN * NT;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv / WN, wn = wv % WN;
    const int Q = o.Q, gi = lane >> 4, li = lane & 15;
    const int64_t g = blockIdx.x;
    const int64_t wo = (g / (8 * nchunk)) * 8 + g % 8;
    const int ch = (int)((g / 8) % nchunk);
    if (wo >= nwork) return;
    const int64_t wi = order[wo];
    if (wi < 0) return;
    const M2LWork wk = work[wi];
    const size_t gper = (size_t)QP * K2, vper = (size_t)NCOL * K2;
    dx4m acc[MT][NT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[a][t] = dx4m{0.0, 0.0, 0.0, 0.0};
    // one step = eight reduction indices of one partner; the operands of the next step
    // are loaded during the products of the current one
    constexpr int KS = K2 / 8;
    const int nstep = (wk.end - wk.beg) * KS;
    double2 av[MT], bv[NT];
    auto load = [&](int it) {
        const int kp = wk.beg + it / KS, s8 = it % KS;
        const double *Gp = Gd + (size_t)gslot[kp] * gper;
        const double *Vs = Vd + ((size_t)(partner[kp] - cl0) * nchunk + ch) * vper;
        const int kb = 8 * s8 + 2 * gi;
        // real rows [Gr, -Gi], imaginary rows [Gi, Gr] of the stored [Gr | Gi]; kb and
        // 8 s8 lie in the same half (QP is a multiple of 16)
        const bool hi = 8 * s8 >= QP;
        const int ksrc = wm == 0 ? kb : (hi ? kb - QP : kb + QP);
#pragma unroll
        for (int t = 0; t < NT; ++t)
            bv[t] = *reinterpret_cast<const double2 *>(Vs + (size_t)(16 * (wn * NT + t) + li) * K2 + kb);
#pragma unroll
        for (int a = 0; a < MT; ++a)
            av[a] = *reinterpret_cast<const double2 *>(Gp + (size_t)(16 * a + li) * K2 + ksrc);
        return wm == 0 && hi;
    };
    bool neg = nstep > 0 ? load(0) : false;
    for (int it = 0; it < nstep; ++it) {
        double2 ca[MT], cb[NT];
#pragma unroll
        for (int a = 0; a < MT; ++a) ca[a] = neg ? make_double2(-av[a].x, -av[a].y) : av[a];
#pragma unroll
        for (int t = 0; t < NT; ++t) cb[t] = bv[t];
        if (it + 1 < nstep) neg = load(it + 1);
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[a][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[a].x, cb[t].x, acc[a][t], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[a][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[a].y, cb[t].y, acc[a][t], 0, 0, 0);
    }
    // lane holds D[lane/16 + 4 j][lane % 16] of each tile: node m, column n = f rc + jc
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = 16 * (wn * NT + t) + li, f = n / rc, jc = n % rc;
        const int col = ch * rc + jc;
        if (f >= 4 || col >= r) continue;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * a + gi + 4 * j;
                if (m < Qr) {
                    double *dst = reinterpret_cast<double *>(part + (((size_t)wi * 4 + f) * Q + m) * r + col);
                    dst[wm] = acc[a][t][j];
                }
            }
    }
}

// The double-buffered product with the real and the imaginary row tiles of a column
// tile in the same wave: WN waves of NT column tiles each, no two waves loading the
// same right-factor fragments (the kernel above loads each twice, once per row half),
// at the price of twice the left-factor reads from shared memory.
template <int SPLIT, int MT, int WN, int NT>
__global__ __launch_bounds__(64 * WN) void k_m2l_mxr(DevOp o, int r, int rc, int nchunk, int64_t nwork, int Qr, int cl0,
                                                     const int32_t *order, const M2LWork *work,
                                                     const int32_t *partner, const int32_t *gslot, const __bf16 *Gb,
                                                     const __bf16 *Vb, float2 *part)
{
    constexpr int PL = SPLIT == 3 ? 2 : 1;
    constexpr int QP = 16 * MT, K2 = 2 * QP, KS = K2 / 32, LD = K2 + IGE_GPAD;
    constexpr int NTH = 64 * WN, NCOL = 16 * WN * NT;
    constexpr int GCH = PL * QP * K2 / 8;           // 16-byte pieces of one block
    constexpr int GV = (GCH + NTH - 1) / NTH;       // pieces per thread
    constexpr int PPS = (GV + KS - 1) / KS;         // pieces per thread per reduction step
    constexpr size_t BUF = (size_t)PL * QP * LD;    // one staging buffer
    extern __shared__ __bf16 sG[];                  // [2][PL][QP][LD]
    const int tid = threadIdx.x, lane = tid & 63, wn = tid >> 6;
    const int Q = o.Q;   // stride of the partial couplings; Qr rows of them written
    const int64_t g = blockIdx.x;
    const int64_t wo = (g / (8 * nchunk)) * 8 + g % 8;
    const int ch = (int)((g / 8) % nchunk);
    if (wo >= nwork) return;
    const int64_t wi = order[wo];
    if (wi < 0) return;   // padding slot of a launch order
    const M2LWork wk = work[wi];
    if (wk.beg >= wk.end) return;
    const size_t gper = (size_t)PL * QP * K2, vper = (size_t)NCOL * K2;

    auto s_piece = [&](__bf16 *buf, int e, uint4 v) {
        const int pl = e / (QP * K2 / 8), rr = e % (QP * K2 / 8), row = rr / (K2 / 8), k8 = rr % (K2 / 8);
        *reinterpret_cast<uint4 *>(buf + ((size_t)pl * QP + row) * LD + 8 * k8) = v;
    };
    auto b_load = [&](bf8 (&b)[NT][PL], int kp, int s) {
        const __bf16 *Vs = Vb + ((size_t)(partner[kp] - cl0) * nchunk + ch) * PL * vper;
        const int kk = 32 * s + 8 * (lane >> 4);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = 16 * (wn * NT + t) + (lane & 15);
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
                b[t][pl] = *reinterpret_cast<const bf8 *>(Vs + (size_t)pl * vper + (size_t)n * K2 + kk);
        }
    };

    f4 acc[2][MT][NT];   // [real rows, imaginary rows]
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[h][a][t] = f4{0.f, 0.f, 0.f, 0.f};

    {   // first block straight into buffer 0
        const __bf16 *Gp = Gb + (size_t)gslot[wk.beg] * gper;
        for (int e = tid; e < GCH; e += NTH) s_piece(sG, e, *reinterpret_cast<const uint4 *>(Gp + (size_t)8 * e));
    }
    bf8 bcur[NT][PL], bnxt[NT][PL];
    b_load(bcur, wk.beg, 0);
    __syncthreads();
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const __bf16 *cur = sG + (size_t)((kp - wk.beg) & 1) * BUF;
        __bf16 *nxt = sG + (size_t)(((kp - wk.beg) & 1) ^ 1) * BUF;
        const int kq = min(kp + 1, wk.end - 1);
        const __bf16 *Gn = Gb + (size_t)gslot[kq] * gper;
        constexpr bool GEVEN = GCH % NTH == 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            uint4 pc[PPS];
#pragma unroll
            for (int v = 0; v < PPS; ++v) {
                const int e = tid + NTH * (s * PPS + v);
                if (s * PPS + v < GV && (GEVEN || e < GCH)) pc[v] = *reinterpret_cast<const uint4 *>(Gn + (size_t)8 * e);
            }
            if (s + 1 < KS) b_load(bnxt, kp, s + 1);
            else b_load(bnxt, kq, 0);
            const bool hi_half = 32 * s >= QP;
            const int kk = 32 * s + 8 * (lane >> 4);
            // real rows [Gr, -Gi]: columns kk of the stored [Gr | Gi] row, negated in the
            // upper half; imaginary rows [Gi, Gr]: the halves swapped
            const int ksrc[2] = {kk, hi_half ? kk - QP : kk + QP};
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                bf8 ah[2], al[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const __bf16 *row = cur + (size_t)(16 * a + (lane & 15)) * LD + ksrc[h];
                    ah[h] = *reinterpret_cast<const bf8 *>(row);
                    if (SPLIT == 3) al[h] = *reinterpret_cast<const bf8 *>(row + (size_t)QP * LD);
                }
                if (hi_half) {
                    ah[0] = neg_bf8(ah[0]);
                    if (SPLIT == 3) al[0] = neg_bf8(al[0]);
                }
                // the split products go over the tile's 2 NT accumulators in turn, so
                // consecutive instructions never share an accumulator
#pragma unroll
                for (int term = 0; term < (SPLIT == 3 ? 3 : 1); ++term)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            const bf8 &A = term == 2 ? al[h] : ah[h];
                            const bf8 &Bv = term == 1 ? bcur[t][PL - 1] : bcur[t][0];
                            acc[h][a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv, acc[h][a][t], 0, 0, 0);
                        }
            }
#pragma unroll
            for (int v = 0; v < PPS; ++v) {
                const int e = tid + NTH * (s * PPS + v);
                if (s * PPS + v < GV && (GEVEN || e < GCH)) s_piece(nxt, e, pc[v]);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl) bcur[t][pl] = bnxt[t][pl];
        }
        __syncthreads();   // the next block is complete and the current buffer is free
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = 16 * (wn * NT + t) + (lane & 15), f = n / rc, jc = n % rc;
        const int col = ch * rc + jc;
        if (f >= 4 || col >= r) continue;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * a + 4 * (lane >> 4) + j;
                if (m < Qr) {
                    float *dst = reinterpret_cast<float *>(part + (((size_t)wi * 4 + f) * Q + m) * r + col);
                    dst[0] = acc[0][a][t][j];
                    dst[1] = acc[1][a][t][j];
                }
            }
    }
}

}  // namespace

int coupling_qp(int Q) { return 32 * ((Q + 31) / 32); }

void ensure_coupling_bf16(ige_op op, int split)
{
    DBuf<__bf16> &G = split == 3 ? op->d_Gb3 : op->d_Gb1;
    if (G.p || op->nfp == 0) return;
    const DevOp &o = op->view;
    const int pl = split == 3 ? 2 : 1;
    if (!op->mxl.empty()) {   // a degree per level: each level's blocks at its own size
        size_t tot = 0;
        for (const auto &L : op->mxl) tot += (size_t)L.np * 2 * L.Qp * 2 * L.Qp;
        G.alloc(tot * pl);
        for (const auto &L : op->mxl) {
            const int64_t n = L.np * 2 * (int64_t)L.Qp * L.Qp;
            hipLaunchKernelGGL(k_gb_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, op->ctx->stream, o, L.np,
                               op->d_fpair.p + 2 * L.p0, L.Qr, L.Qp, split, G.p + L.gb_off * pl);
            IGE_HIP(hipGetLastError());
        }
        return;
    }
    const int Qp = coupling_qp(o.Q);
    G.alloc((size_t)op->nfp * 2 * pl * Qp * 2 * Qp);
    const int64_t n = op->nfp * 2 * (int64_t)Qp * Qp;
    hipLaunchKernelGGL(k_gb_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, op->ctx->stream, o, op->nfp,
                       op->d_fpair.p, o.Q, Qp, split, G.p);
    IGE_HIP(hipGetLastError());
}

namespace {

// columns per chunk (complex columns = 4 fields x right-hand sides): the smallest of
// 16..256 holding all 4r columns, capped so that the accumulators, the prefetched
// block and the streamed factor stay in registers (no spills)
// double-buffered staging: both buffers fit in shared memory (64 KB is the limit for
// dynamic shared memory granted without asking; up to 160 KB after the attribute)
bool m2l_db_fits(int MT, int split) { return (size_t)2 * (split == 3 ? 2 : 1) * 16 * MT * (32 * MT + IGE_GPAD) * 2 <= 160 * 1024; }

// widest chunk (complex columns) without register spills; db: double-buffered kernel
int m2l_ncol_cap(int MT, int split, bool db)
{
    if (db) return MT >= 8 ? 128 : 256;
    return MT >= 8 ? (split == 3 ? 64 : 128) : (MT >= 6 ? 128 : 256);
}

// the smallest of 16..cap holding all 4r columns
int m2l_ncol(int r, int cap)
{
    int nc = 16;
    while (nc < 4 * r && nc < cap) nc *= 2;
    return nc;
}

// the work items of one launch: their launch order (nw entries, -1 = padding), the
// rows of their blocks and the first cluster of their level (the right factors of
// that level start there)
struct MxSpan {
    const int32_t *order;
    int64_t nw;
    int Qr, cl0;
};

template <bool DB, int SPLIT, int MT, int WN, int NT>
void launch_mx(ige_op op, int r, int rc, int nchunk, const __bf16 *G, const __bf16 *Vb, hipStream_t s,
               const MxSpan &sp)
{
    const DevOp &o = op->view;
    const int64_t nw = sp.nw;
    const int32_t *order = sp.order;
    const dim3 grid((unsigned)(((nw + 7) / 8) * 8 * nchunk)), blk(128 * WN);
    constexpr int PL = SPLIT == 3 ? 2 : 1, QP = 16 * MT;
    constexpr size_t shm = sizeof(__bf16) * (DB ? 2 : 1) * PL * QP * (2 * QP + IGE_GPAD);
    auto kern = DB ? &k_m2l_mxd<SPLIT, MT, WN, NT> : &k_m2l_mx<SPLIT, MT, WN, NT>;
    // the attribute is set once per kernel (thread-safe static initialisation; a throw
    // leaves it unset for the next call), before any graph capture
    static const bool attr = [&] {
        int lds_max = 0;
        IGE_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, op->ctx->device));
        IGE_REQUIRE(shm <= (size_t)lds_max, "coupling block does not fit in shared memory");
        IGE_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm));
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(kern, grid, blk, shm, s, o, r, rc, nchunk, nw, sp.Qr, sp.cl0, order, op->d_mwork.p,
                       op->d_mpartner.p, op->d_gslot.p, G, Vb, op->d_bmpart.p);
    IGE_HIP(hipGetLastError());
}

// the rows-merged kernel (k_m2l_mxr): WN waves of NT column tiles
template <int SPLIT, int MT, int WN, int NT>
void launch_mxr(ige_op op, int r, int rc, int nchunk, const __bf16 *G, const __bf16 *Vb, hipStream_t s,
                const MxSpan &sp)
{
    const DevOp &o = op->view;
    const int64_t nw = sp.nw;
    const int32_t *order = sp.order;
    const dim3 grid((unsigned)(((nw + 7) / 8) * 8 * nchunk)), blk(64 * WN);
    constexpr int PL = SPLIT == 3 ? 2 : 1, QP = 16 * MT;
    constexpr size_t shm = sizeof(__bf16) * 2 * PL * QP * (2 * QP + IGE_GPAD);
    auto kern = &k_m2l_mxr<SPLIT, MT, WN, NT>;
    static const bool attr = [&] {
        int lds_max = 0;
        IGE_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, op->ctx->device));
        IGE_REQUIRE(shm <= (size_t)lds_max, "coupling block does not fit in shared memory");
        IGE_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm));
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(kern, grid, blk, shm, s, o, r, rc, nchunk, nw, sp.Qr, sp.cl0, order, op->d_mwork.p,
                       op->d_mpartner.p, op->d_gslot.p, G, Vb, op->d_bmpart.p);
    IGE_HIP(hipGetLastError());
}

template <bool DB, int SPLIT, int MT>
void launch_mx_cols(ige_op op, int r, int ncol, const __bf16 *G, const __bf16 *Vb, hipStream_t s, const MxSpan &sp)
{
    const int rc = ncol / 4, nchunk = (r + rc - 1) / rc;
    // wide double-buffered chunks: the rows-merged kernel (IGE_M2L_RM=0 keeps the other)
    if constexpr (DB) {
        if (op->m2l_rm && ncol == 256 && MT <= 6) {
            launch_mxr<SPLIT, MT, 8, 2>(op, r, rc, nchunk, G, Vb, s, sp);
            return;
        }
        if (op->m2l_rm && ncol == 128) {
            launch_mxr<SPLIT, MT, 8, 1>(op, r, rc, nchunk, G, Vb, s, sp);
            return;
        }
    }
    switch (ncol) {
        case 16: launch_mx<DB, SPLIT, MT, 1, 1>(op, r, rc, nchunk, G, Vb, s, sp); break;
        case 32: launch_mx<DB, SPLIT, MT, 2, 1>(op, r, rc, nchunk, G, Vb, s, sp); break;
        case 64: launch_mx<DB, SPLIT, MT, 4, 1>(op, r, rc, nchunk, G, Vb, s, sp); break;
        case 128:
            if constexpr (DB || SPLIT == 1 || MT < 8) launch_mx<DB, SPLIT, MT, 4, 2>(op, r, rc, nchunk, G, Vb, s, sp);
            else IGE_REQUIRE(false, "coupling chunk too wide for this interpolation degree");
            break;
        default:
            if constexpr (MT <= 4 || (DB && MT <= 6)) launch_mx<DB, SPLIT, MT, 4, 4>(op, r, rc, nchunk, G, Vb, s, sp);
            else IGE_REQUIRE(false, "coupling chunk too wide for this interpolation degree");
            break;
    }
}

template <bool DB, int SPLIT>
void launch_mx_mt(ige_op op, int r, int MT, int ncol, const __bf16 *G, const __bf16 *Vb, hipStream_t s,
                  const MxSpan &sp)
{
    switch (MT) {
        case 2: launch_mx_cols<DB, SPLIT, 2>(op, r, ncol, G, Vb, s, sp); break;
        case 4: launch_mx_cols<DB, SPLIT, 4>(op, r, ncol, G, Vb, s, sp); break;
        case 6: launch_mx_cols<DB, SPLIT, 6>(op, r, ncol, G, Vb, s, sp); break;
        default:
            if constexpr (!DB || SPLIT == 1) launch_mx_cols<DB, SPLIT, 8>(op, r, ncol, G, Vb, s, sp);
            else IGE_REQUIRE(false, "double-buffered coupling blocks do not fit in shared memory");
            break;
    }
}

}  // namespace

int m2l_ncol_limit(ige_op op, int r, int split)
{
    int Qp = coupling_qp(op->view.Q);
    if (!op->mxl.empty()) {
        Qp = 0;
        for (const auto &L : op->mxl) Qp = std::max(Qp, L.Qp);
    }
    const int MT = Qp / 16;
    const bool db = m2l_db_fits(MT, split) && tune_get(op, kTuneM2lDb, r, split, 1) != 0;
    return m2l_ncol_cap(MT, split, db);
}

namespace {
// the right factor of clusters cl0 .. cl0 + ncl - 1 (Qr nodes each) for one chunking
void vb_prep(ige_op op, int cl0, int ncl, int Qr, int r, int rc, int nchunk, int ncol, int Qp, int split,
             const double2 *src, __bf16 *Vb, hipStream_t s)
{
    const DevOp &o = op->view;
    if (rc <= 64) {   // every element of the chunk's right factor is written (zeros in the padding)
        const int64_t nb = (int64_t)ncl * nchunk * 4 * (Qp / kVbRows);
        hipLaunchKernelGGL(k_vb_prep_t, dim3((unsigned)nb), dim3(256), 0, s, o, cl0, Qr, r, rc, nchunk, ncol, Qp, split,
                           src, Vb);
    } else {
        const int64_t nv = (int64_t)ncl * nchunk * ncol * 2 * Qp;
        hipLaunchKernelGGL(k_vb_prep, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, o, ncl, cl0, Qr, r, rc,
                           nchunk, ncol, Qp, split, src, Vb);
    }
    IGE_HIP(hipGetLastError());
}

void mx_run(ige_op op, int r, int split, bool db, int MT, int ncol, const __bf16 *G, const __bf16 *Vb, hipStream_t s,
            const MxSpan &sp)
{
    if (db) {
        if (split == 3) launch_mx_mt<true, 3>(op, r, MT, ncol, G, Vb, s, sp);
        else launch_mx_mt<true, 1>(op, r, MT, ncol, G, Vb, s, sp);
    } else {
        if (split == 3) launch_mx_mt<false, 3>(op, r, MT, ncol, G, Vb, s, sp);
        else launch_mx_mt<false, 1>(op, r, MT, ncol, G, Vb, s, sp);
    }
}

// a degree per level: per level its padded block size, chunking and launch
void m2l_bf16_levels(ige_op op, int r, int split, const double2 *src, hipStream_t s, hipEvent_t mid)
{
    const DevOp &o = op->view;
    const int planes = split == 3 ? 2 : 1;
    const __bf16 *G = split == 3 ? op->d_Gb3.p : op->d_Gb1.p;
    struct Plan {
        int MT, ncol, rc, nchunk;
        bool db;
        size_t vb_off;
    };
    std::vector<Plan> pl(op->mxl.size());
    size_t vbn = 0;
    for (size_t i = 0; i < op->mxl.size(); ++i) {
        const auto &L = op->mxl[i];
        Plan &P = pl[i];
        P.MT = L.Qp / 16;
        IGE_REQUIRE(P.MT <= 8, "interpolation degree too large for the matrix-core coupling");
        P.db = m2l_db_fits(P.MT, split);
        P.ncol = m2l_ncol(r, m2l_ncol_cap(P.MT, split, P.db));
        P.rc = P.ncol / 4;
        P.nchunk = (r + P.rc - 1) / P.rc;
        P.vb_off = vbn;
        vbn += (size_t)L.ncl * P.nchunk * planes * P.ncol * 2 * L.Qp;
    }
    if (op->d_vb.n < vbn) op->d_vb.alloc(vbn);
    const size_t pn = op->mwork.size() * 4 * (size_t)o.Q * r;
    if (op->d_bmpart.n < pn) op->d_bmpart.alloc(pn);
    for (size_t i = 0; i < op->mxl.size(); ++i) {
        const auto &L = op->mxl[i];
        vb_prep(op, L.cl0, L.ncl, L.Qr, r, pl[i].rc, pl[i].nchunk, pl[i].ncol, L.Qp, split, src,
                op->d_vb.p + pl[i].vb_off, s);
    }
    if (mid) IGE_HIP(hipEventRecord(mid, s));
    for (size_t i = 0; i < op->mxl.size(); ++i) {
        const auto &L = op->mxl[i];
        const MxSpan sp{op->d_morder.p + L.w0, L.nw, L.Qr, L.cl0};
        mx_run(op, r, split, pl[i].db, pl[i].MT, pl[i].ncol, G + L.gb_off * planes, op->d_vb.p + pl[i].vb_off, s, sp);
    }
}
}  // namespace

void m2l_bf16(ige_op op, int r, int split, const double2 *src, hipStream_t s, hipEvent_t mid)
{
    const DevOp &o = op->view;
    if (op->mwork.empty()) return;
    ensure_coupling_bf16(op, split);
    if (!op->mxl.empty()) {
        m2l_bf16_levels(op, r, split, src, s, mid);
        return;
    }
    const int Qp = coupling_qp(o.Q), K2 = 2 * Qp, MT = Qp / 16;
    IGE_REQUIRE(MT <= 8, "interpolation degree too large for the matrix-core coupling");
    // staging (single or double buffer) and chunk width: tuned values if any, else
    // double-buffered where it fits and the smallest chunk holding all columns
    const bool db = m2l_db_fits(MT, split) && tune_get(op, kTuneM2lDb, r, split, 1) != 0;
    const int cap = m2l_ncol_cap(MT, split, db);
    int ncol = m2l_ncol(r, cap);
    const int tuned = tune_get(op, kTuneM2lNcol, r, split, 0);
    if (tuned >= 16 && (tuned & (tuned - 1)) == 0) ncol = std::min(tuned, cap);
    const int rc = ncol / 4, nchunk = (r + rc - 1) / rc;
    const int planes = split == 3 ? 2 : 1;
    const size_t vbn = (size_t)op->NC * nchunk * planes * ncol * K2;
    if (op->d_vb.n < vbn) op->d_vb.alloc(vbn);
    const size_t pn = op->mwork.size() * 4 * (size_t)o.Q * r;
    if (op->d_bmpart.n < pn) op->d_bmpart.alloc(pn);
    vb_prep(op, 0, op->NC, o.Q, r, rc, nchunk, ncol, Qp, split, src, op->d_vb.p, s);
    if (mid) IGE_HIP(hipEventRecord(mid, s));
    // launch order: decreasing partner count (default) or cluster order per XCD
    const bool spatial = tune_get(op, kTuneM2lOrder, r, split, 0) == 1 && op->n_morder_sp > 0;
    const MxSpan sp{spatial ? op->d_morder_sp.p : op->d_morder.p, spatial ? op->n_morder_sp : (int64_t)op->mwork.size(),
                    o.Q, 0};
    mx_run(op, r, split, db, MT, ncol, split == 3 ? op->d_Gb3.p : op->d_Gb1.p, op->d_vb.p, s, sp);
}


namespace {
template <int MT, int WN, int NT>
void launch_md(ige_op op, int r, int rc, int nchunk, hipStream_t s, const MxSpan &sp, const double *Gd,
               const double *Vd)
{
    const DevOp &o = op->view;
    const int64_t nw = sp.nw;
    const dim3 grid((unsigned)(((nw + 7) / 8) * 8 * nchunk)), blk(128 * WN);
    hipLaunchKernelGGL((k_m2l_md<MT, WN, NT>), grid, blk, 0, s, o, r, rc, nchunk, nw, sp.Qr, sp.cl0, sp.order,
                       op->d_mwork.p, op->d_mpartner.p, op->d_gslot.p, Gd, Vd, op->d_bmpart64.p);
    IGE_HIP(hipGetLastError());
}

template <int MT>
void launch_md_cols(ige_op op, int r, int ncol, hipStream_t s, const MxSpan &sp, const double *Gd, const double *Vd)
{
    const int rc = ncol / 4, nchunk = (r + rc - 1) / rc;
    switch (ncol) {
        case 16: launch_md<MT, 1, 1>(op, r, rc, nchunk, s, sp, Gd, Vd); break;
        case 32: launch_md<MT, 2, 1>(op, r, rc, nchunk, s, sp, Gd, Vd); break;
        case 64: launch_md<MT, 4, 1>(op, r, rc, nchunk, s, sp, Gd, Vd); break;
        default: launch_md<MT, 4, 2>(op, r, rc, nchunk, s, sp, Gd, Vd); break;
    }
}

void md_run(ige_op op, int r, int MT, int ncol, hipStream_t s, const MxSpan &sp, const double *Gd, const double *Vd)
{
    switch (MT) {
        case 2: launch_md_cols<2>(op, r, ncol, s, sp, Gd, Vd); break;
        case 4: launch_md_cols<4>(op, r, ncol, s, sp, Gd, Vd); break;
        case 6: launch_md_cols<6>(op, r, ncol, s, sp, Gd, Vd); break;
        default: launch_md_cols<8>(op, r, ncol, s, sp, Gd, Vd); break;
    }
}

// the FP64 blocks of one level (or of all levels at one degree) and their size
size_t gd_count(int64_t np, int Qp) { return (size_t)np * 2 * Qp * 2 * Qp; }
}  // namespace

void ensure_coupling_f64(ige_op op)
{
    if (op->d_Gd.p || op->nfp == 0) return;
    const DevOp &o = op->view;
    if (!op->mxl.empty()) {   // a degree per level: each level's blocks at its own size
        size_t tot = 0;
        for (const auto &L : op->mxl) tot += gd_count(L.np, L.Qp);
        op->d_Gd.alloc(tot);
        size_t off = 0;
        for (const auto &L : op->mxl) {
            const int64_t n = L.np * 2 * (int64_t)L.Qp * L.Qp;
            hipLaunchKernelGGL(k_gd_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, op->ctx->stream, o, L.np,
                               op->d_fpair.p + 2 * L.p0, L.Qr, L.Qp, op->d_Gd.p + off);
            IGE_HIP(hipGetLastError());
            off += gd_count(L.np, L.Qp);
        }
        return;
    }
    const int Qp = coupling_qp(o.Q);
    op->d_Gd.alloc(gd_count(op->nfp, Qp));
    const int64_t n = op->nfp * 2 * (int64_t)Qp * Qp;
    hipLaunchKernelGGL(k_gd_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, op->ctx->stream, o, op->nfp,
                       op->d_fpair.p, o.Q, Qp, op->d_Gd.p);
    IGE_HIP(hipGetLastError());
}

bool m2l_f64mx_ok(ige_op op, int r)
{
    if (r < 8 || op->mwork.empty() || op->f64mx_off) return false;
    size_t need = 0;
    if (!op->mxl.empty()) {   // a degree per level: every level's blocks within 128 padded nodes
        for (const auto &L : op->mxl) {
            if (L.Qp > 128) return false;
            need += gd_count(L.np, L.Qp) * sizeof(double);
        }
    } else {
        const int Qp = coupling_qp(op->view.Q);
        if (Qp > 128) return false;
        need = gd_count(op->nfp, Qp) * sizeof(double);
    }
    if (op->gd_fit < 0) {   // decided once, at the first eligible apply (never under capture)
        size_t fr = 0, tot = 0;
        IGE_HIP(hipMemGetInfo(&fr, &tot));
        op->gd_fit = op->d_Gd.p || need + ((size_t)8 << 30) < fr ? 1 : 0;
    }
    return op->gd_fit == 1;
}

bool m2l_f64mx_use(ige_op op, int r) { return m2l_f64mx_ok(op, r) && tune_get(op, kTuneM2lF64, r, IGE_F64, 1) != 0; }

void m2l_f64mx(ige_op op, int r, const double2 *src, hipStream_t s, hipEvent_t mid)
{
    const DevOp &o = op->view;
    if (op->mwork.empty()) return;
    ensure_coupling_f64(op);
    int ncol = 16;
    while (ncol < 4 * r && ncol < 128) ncol *= 2;
    const int rc = ncol / 4, nchunk = (r + rc - 1) / rc;
    const size_t pn = op->mwork.size() * 4 * (size_t)o.Q * r;
    if (op->d_bmpart64.n < pn) op->d_bmpart64.alloc(pn);
    if (!op->mxl.empty()) {   // level by level, each with its padded block size
        size_t vdn = 0;
        for (const auto &L : op->mxl) vdn += (size_t)L.ncl * nchunk * ncol * 2 * L.Qp;
        if (op->d_vd.n < vdn) op->d_vd.alloc(vdn);
        size_t voff = 0;
        std::vector<size_t> vo(op->mxl.size());
        for (size_t i = 0; i < op->mxl.size(); ++i) {
            const auto &L = op->mxl[i];
            vo[i] = voff;
            const int64_t nb = (int64_t)L.ncl * nchunk * 4 * (L.Qp / kVbRows);
            hipLaunchKernelGGL(k_vd_prep_t, dim3((unsigned)nb), dim3(256), 0, s, o, L.cl0, L.Qr, r, rc, nchunk, ncol,
                               L.Qp, src, op->d_vd.p + voff);
            IGE_HIP(hipGetLastError());
            voff += (size_t)L.ncl * nchunk * ncol * 2 * L.Qp;
        }
        if (mid) IGE_HIP(hipEventRecord(mid, s));
        size_t goff = 0;
        for (size_t i = 0; i < op->mxl.size(); ++i) {
            const auto &L = op->mxl[i];
            IGE_REQUIRE(L.Qp / 16 <= 8, "interpolation degree too large for the matrix-core coupling");
            const MxSpan sp{op->d_morder.p + L.w0, L.nw, L.Qr, L.cl0};
            md_run(op, r, L.Qp / 16, ncol, s, sp, op->d_Gd.p + goff, op->d_vd.p + vo[i]);
            goff += gd_count(L.np, L.Qp);
        }
        return;
    }
    const int Qp = coupling_qp(o.Q), K2 = 2 * Qp, MT = Qp / 16;
    IGE_REQUIRE(MT <= 8, "interpolation degree too large for the matrix-core coupling");
    const size_t vdn = (size_t)op->NC * nchunk * ncol * K2;
    if (op->d_vd.n < vdn) op->d_vd.alloc(vdn);
    const int64_t nb = (int64_t)op->NC * nchunk * 4 * (Qp / kVbRows);
    hipLaunchKernelGGL(k_vd_prep_t, dim3((unsigned)nb), dim3(256), 0, s, o, 0, o.Q, r, rc, nchunk, ncol, Qp, src,
                       op->d_vd.p);
    IGE_HIP(hipGetLastError());
    if (mid) IGE_HIP(hipEventRecord(mid, s));
    const MxSpan sp{op->d_morder.p, (int64_t)op->mwork.size(), o.Q, 0};
    md_run(op, r, MT, ncol, s, sp, op->d_Gd.p, op->d_vd.p);
}

}  // namespace ige
