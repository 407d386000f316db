// Coupling stage (a5) on the BF16 matrix cores, for many right-hand sides.
//
// The kernel matrices G of the admissible pairs are stored once in BF16, in both
// orientations (G_ts row-major and G_st = G_ts^T row-major), so that the operand of
// every ordered pair t <- s has its reduction index contiguous.  A complex product
// U_t = G_ts V_s is one real product
//   [Re U | Im U] (interleaved per column) = [Gr | Gi] (Qp x 2Qp) . [[Vr, Vi], [-Vi, Vr]]
// with FP32 accumulation on the 16x16x32 BF16 instruction (lane l supplies
// A[l%16][8(l/16)+i] and B[8(l/16)+i][l%16]; accumulator register j of lane l holds
// D[4(l/16)+j][l%16]).  With split = 3 both factors are stored as a BF16 pair
// (x = xh + xl) and the product is xh.yh + xh.yl + xl.yh (about 2^-16 relative).
//
// Work: one workgroup per (target cluster, up to 32 partners, 8 right-hand sides);
// the source fields are converted once per apply into the operand layout; partial
// couplings per work item are summed by the fixed-order per-cluster reduction.
#include <hip/hip_runtime.h>

#include "device_math.hpp"
#include "op.hpp"

namespace ige {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kRC = 8;            // right-hand sides per column chunk
constexpr int kNCol = 8 * kRC;    // real operand columns per chunk: 4 fields x kRC x (re, im)

__device__ inline void split_bf16(double x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)(float)x;
    lo = (__bf16)(float)(x - (double)(float)hi);
}

// G in BF16: Gb[(2 pair + orientation) * planes + plane][Qp][2Qp] (planes = 2 for the
// split form: high and low part, else 1); orientation 0 =
// G_ts (rows: nodes of t), 1 = G_st; columns [Re | Im], zero padded
__global__ void k_gb_store(DevOp o, int64_t nfp, const int32_t *fpair, int Qp, int split, __bf16 *Gb)
{
    const int Q = o.Q, K2 = 2 * Qp;
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
        const double *Xa = o.nodeX + (size_t)ga * 3 * Q, *Xb = o.nodeX + (size_t)gb * 3 * Q;
        const double d0 = Xa[m] - Xb[mc], d1 = Xa[Q + m] - Xb[Q + mc], d2 = Xa[2 * Q + m] - Xb[2 * Q + mc];
        g = dm::helmholtz_r2(o.kappa, fma(d0, d0, fma(d1, d1, d2 * d2)));
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

// Source fields [NC][4][Q][r] -> operand layout Vb[cluster][chunk][plane][kNCol][2Qp]
// (planes as for G):
// column n = 2 c + h (c = field * kRC + column in chunk, h = re/im), row k:
// k < Qp: (Vr, Vi)[k], k >= Qp: (-Vi, Vr)[k - Qp]
__global__ void k_vb_prep(DevOp o, int NC, int r, int nchunk, int Qp, int split, const double2 *src, __bf16 *Vb)
{
    const int Q = o.Q, K2 = 2 * Qp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)kNCol * K2;
    if (t >= (int64_t)NC * nchunk * per) return;
    const int64_t cc = t / per;   // cluster * nchunk + chunk
    const int rem = (int)(t % per), n = rem / K2, k = rem % K2;
    const int gc = (int)(cc / nchunk), ch = (int)(cc % nchunk);
    const int c = n >> 1, h = n & 1, f = c / kRC, j = c % kRC, col = ch * kRC + j;
    const int mm = k < Qp ? k : k - Qp;
    double v = 0.0;
    if (mm < Q && col < r) {
        const double2 s = src[(((size_t)gc * 4 + f) * Q + mm) * r + col];
        v = k < Qp ? (h ? s.y : s.x) : (h ? s.x : -s.y);
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

// 4 waves as 2 (row halves) x 2 (column halves); a wave holds MT row tiles x 2 column
// tiles of the Qp x kNCol output
template <int MT, int SPLIT>
__global__ __launch_bounds__(256) void k_m2l_bf16(DevOp o, int r, int nchunk, int64_t nwork, int Qp,
                                                  const M2LWork *work, const int32_t *partner, const int32_t *gslot,
                                                  const __bf16 *Gb, const __bf16 *Vb, double2 *part)
{
    constexpr int PL = SPLIT == 3 ? 2 : 1;   // BF16 planes per operand
    extern __shared__ __bf16 sV[];   // [PL][kNCol][K2 + 8]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
    const int Q = o.Q, K2 = 2 * Qp, KS = K2 / 32, QT = Qp / 16, LD = K2 + 8;
    // the chunks of one work item share an XCD (consecutive ids go round-robin over 8)
    const int64_t g = blockIdx.x;
    const int64_t wi = (g / (8 * nchunk)) * 8 + g % 8;
    const int ch = (int)((g / 8) % nchunk);
    if (wi >= nwork) return;
    const M2LWork wk = work[wi];
    f4 acc[MT][2];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    const size_t vper = (size_t)kNCol * K2;
    for (int kp = wk.beg; kp < wk.end; ++kp) {
        const int sc = partner[kp];
        const __bf16 *Vs = Vb + ((size_t)sc * nchunk + ch) * PL * vper;
        __syncthreads();
        // stage the source operand (16-byte pieces) into shared memory
        for (int e = threadIdx.x; e < PL * kNCol * K2 / 8; e += blockDim.x) {
            const int pl = e / (kNCol * K2 / 8), rr = e % (kNCol * K2 / 8), n = rr / (K2 / 8), k8 = rr % (K2 / 8);
            *reinterpret_cast<bf8 *>(sV + ((size_t)pl * kNCol + n) * LD + 8 * k8) =
                *reinterpret_cast<const bf8 *>(Vs + (size_t)pl * vper + (size_t)n * K2 + 8 * k8);
        }
        __syncthreads();
        const __bf16 *Gp = Gb + (size_t)gslot[kp] * PL * Qp * K2;
        for (int s = 0; s < KS; ++s) {
            const int kk = 32 * s + 8 * (lane >> 4);
            bf8 bh[2], bl[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int n = 16 * (2 * wn + b) + (lane & 15);
                bh[b] = *reinterpret_cast<const bf8 *>(sV + (size_t)n * LD + kk);
                if (SPLIT == 3) bl[b] = *reinterpret_cast<const bf8 *>(sV + ((size_t)kNCol + n) * LD + kk);
            }
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const int mt = wm * MT + a;
                if (mt >= QT) break;   // uniform over the wave
                const size_t ro = (size_t)(16 * mt + (lane & 15)) * K2 + kk;
                const bf8 ah = *reinterpret_cast<const bf8 *>(Gp + ro);
                bf8 al;
                if (SPLIT == 3) al = *reinterpret_cast<const bf8 *>(Gp + (size_t)Qp * K2 + ro);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[b], acc[a][b], 0, 0, 0);
                    if (SPLIT == 3) {
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[b], acc[a][b], 0, 0, 0);
                    }
                }
            }
        }
    }
    // lane holds D[4 (lane/16) + j][lane % 16] of each tile: row m, column n = 2 c + h
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        const int mt = wm * MT + a;
        if (mt >= QT) break;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int n = 16 * (2 * wn + b) + (lane & 15), c = n >> 1, h = n & 1, f = c / kRC, jc = c % kRC;
            const int col = ch * kRC + jc;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * mt + 4 * (lane >> 4) + j;
                if (m < Q && col < r) {
                    double *dst = reinterpret_cast<double *>(part + (((size_t)wi * 4 + f) * Q + m) * r + col);
                    dst[h] = (double)acc[a][b][j];
                }
            }
        }
    }
}

}  // namespace

int coupling_qp(int Q) { return 16 * ((Q + 15) / 16); }

void ensure_coupling_bf16(ige_op op, int split)
{
    DBuf<__bf16> &G = split == 3 ? op->d_Gb3 : op->d_Gb1;
    if (G.p || op->nfp == 0) return;
    const DevOp &o = op->view;
    const int Qp = coupling_qp(o.Q);
    G.alloc((size_t)op->nfp * 2 * (split == 3 ? 2 : 1) * Qp * 2 * Qp);
    const int64_t n = op->nfp * 2 * (int64_t)Qp * Qp;
    hipLaunchKernelGGL(k_gb_store, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, op->ctx->stream, o, op->nfp,
                       op->d_fpair.p, Qp, split, G.p);
    IGE_HIP(hipGetLastError());
}

namespace {
template <int SPLIT>
void launch_m2l_bf16_mt(ige_op op, int r, int nchunk, int MT, const __bf16 *G, const __bf16 *Vb, size_t shm)
{
    const DevOp &o = op->view;
    const int64_t nw = (int64_t)op->mwork.size();
    const dim3 grid((unsigned)(((nw + 7) / 8) * 8 * nchunk)), blk(256);
    hipStream_t s = op->ctx->stream;
    const int Qp = coupling_qp(o.Q);
#define IGE_BF16_CASE(M)                                                                                            \
    case M:                                                                                                         \
        hipLaunchKernelGGL((k_m2l_bf16<M, SPLIT>), grid, blk, shm, s, o, r, nchunk, nw, Qp, op->d_mwork.p,          \
                           op->d_mpartner.p, op->d_gslot.p, G, Vb, op->d_bmpart.p);                                 \
        break;
    switch (MT) {
        IGE_BF16_CASE(1)
        IGE_BF16_CASE(2)
        IGE_BF16_CASE(3)
        IGE_BF16_CASE(4)
        default: IGE_BF16_CASE(5)
    }
#undef IGE_BF16_CASE
    IGE_HIP(hipGetLastError());
}
}  // namespace

void m2l_bf16(ige_op op, int r, int split, const double2 *src, hipStream_t s)
{
    const DevOp &o = op->view;
    if (op->mwork.empty()) return;
    ensure_coupling_bf16(op, split);
    const int Qp = coupling_qp(o.Q), K2 = 2 * Qp, QT = Qp / 16, MT = (QT + 1) / 2;
    IGE_REQUIRE(MT <= 5, "interpolation degree too large for the matrix-core coupling");
    const int nchunk = (r + kRC - 1) / kRC;
    const int planes = split == 3 ? 2 : 1;
    const size_t vbn = (size_t)op->NC * nchunk * planes * kNCol * K2;
    if (op->d_vb.n < vbn) op->d_vb.alloc(vbn);
    const size_t pn = op->mwork.size() * 4 * (size_t)o.Q * r;
    if (op->d_bmpart.n < pn) op->d_bmpart.alloc(pn);
    const int64_t nv = (int64_t)op->NC * nchunk * kNCol * K2;
    hipLaunchKernelGGL(k_vb_prep, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, o, op->NC, r, nchunk, Qp,
                       split, src, op->d_vb.p);
    IGE_HIP(hipGetLastError());
    const size_t shm = sizeof(__bf16) * planes * kNCol * (K2 + 8);
    if (split == 3) launch_m2l_bf16_mt<3>(op, r, nchunk, MT, op->d_Gb3.p, op->d_vb.p, shm);
    else launch_m2l_bf16_mt<1>(op, r, nchunk, MT, op->d_Gb1.p, op->d_vb.p, shm);
}

}  // namespace ige
