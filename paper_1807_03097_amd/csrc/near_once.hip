// Near-field product of one column over the distinct entries of the symmetric
// near-field matrix (Sec. 4.2: the non-admissible blocks carry the exact Galerkin
// entries of Sec. 4.1, and the matrix is complex symmetric).  The entries are stored
// once, in dense rectangles of owner blocks (see NearCompact in setup.hpp); the
// values are summed at assembly from the leaf-pair blocks (k_near_merge).  The
// product writes per-rectangle row and column sums, which the fixed-order gather of
// kernels.hip adds per unknown, so the result does not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.hpp"
#include "op.hpp"

namespace ige {

namespace {

typedef double d2v __attribute__((ext_vector_type(2)));

// streaming load of one complex entry (not kept in the caches)
__device__ inline d2v ld_once(const double2 *B, size_t i)
{
    return __builtin_nontemporal_load(reinterpret_cast<const d2v *>(B) + i);
}

// ---------------------------------------------------------------------------
// a8, once per distinct entry: a workgroup streams rows [r0, r1) of one dense
// rectangle of the symmetric near-field matrix (rows and columns are lists of glued
// unknowns); each row gives its row sum (B x_cols)[r] and the same loads give the
// column sums of B^T x_rows.  A diagonal square is read in its upper triangle only:
// row r takes the columns c >= r for its row sum and c > r for the column sums.
// ---------------------------------------------------------------------------
constexpr int kCmpRows = 128;   // largest rows per work item (host: rows_per_item)

template <int U, int RS, int PRIO>
__device__ __forceinline__ void near_cmp_item(const NearCmpView &v, int w, const double2 *x, double2 *part,
                                              double2 *sxr, double2 (*syc)[256])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int4 it = v.work[w];
    const int k = it.x, r0 = it.y, r1 = it.z;
    const int nr = v.nr[k], nc = v.nc[k], ld = v.ld[k];
    const bool sym = v.sym[k] != 0;
    const int32_t *rows = v.idx + v.lst[k], *cols = rows + nr;
    const double2 *B = v.val + v.val_off[k];
    d2v xc[U], yc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int c = lane + 64 * u;
        const double2 xv = c < nc ? x[cols[c]] : make_double2(0.0, 0.0);
        xc[u] = d2v{xv.x, xv.y};
        yc[u] = d2v{0.0, 0.0};
    }
    for (int q = threadIdx.x; q < r1 - r0; q += blockDim.x) sxr[q] = x[rows[r0 + q]];
    __syncthreads();
    if constexpr (PRIO > 0) __builtin_amdgcn_s_setprio(PRIO);
    for (int r = r0 + wv; r < r1; r += 4 * RS) {
        d2v al[RS][U];
#pragma unroll
        for (int q = 0; q < RS; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lane + 64 * u, rq = r + 4 * q;
                al[q][u] = (c < nc && rq < r1 && (!sym || c >= rq)) ? ld_once(B, (size_t)rq * ld + c) : d2v{0.0, 0.0};
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
            const int c = lane + 64 * u;
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const d2v a = al[q][u];
                re[q] = fma(a.x, xc[u].x, fma(-a.y, xc[u].y, re[q]));
                im[q] = fma(a.x, xc[u].y, fma(a.y, xc[u].x, im[q]));
            }
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                // the diagonal entry of a square counts once (row sum only)
                const d2v a = (sym && c == r + 4 * q) ? d2v{0.0, 0.0} : al[q][u];
                yc[u].x = fma(a.x, xq[q].x, fma(-a.y, xq[q].y, yc[u].x));
                yc[u].y = fma(a.x, xq[q].y, fma(a.y, xq[q].x, yc[u].y));
            }
        }
        double vv[2 * RS];
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            vv[2 * q] = re[q];
            vv[2 * q + 1] = im[q];
        }
        const double tot = dm::Halve<2 * RS>::run(vv, lane, 32);
        constexpr int SH = 6 - dm::log2c<2 * RS>();
        if ((lane & ((1 << SH) - 1)) == 0) {
            const int kk = lane >> SH;   // value 2 q + (0: real, 1: imaginary part)
            const int rq = r + 4 * (kk >> 1);
            if (rq < r1) reinterpret_cast<double *>(part)[2 * (v.wpart[w] + (rq - r0)) + (kk & 1)] = tot;
        }
    }
    if (wv > 0)
#pragma unroll
        for (int u = 0; u < U; ++u) syc[wv - 1][lane + 64 * u] = make_double2(yc[u].x, yc[u].y);
    __syncthreads();
    if (wv == 0) {
        double2 *cp = part + v.wpart[w] + (r1 - r0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = lane + 64 * u;
            if (c < nc) {
                const double2 s1 = syc[0][c], s2 = syc[1][c], s3 = syc[2][c];
                cp[c] = make_double2(((yc[u].x + s1.x) + s2.x) + s3.x, ((yc[u].y + s1.y) + s2.y) + s3.y);
            }
        }
    }
}

// Work items of at most 128 columns take two column groups of 64 per lane; the wider
// ones U of them, in a second launch (obase: first item of the launch in the order).
template <int U, int RS, int PRIO>
__global__ __launch_bounds__(256) void k_near_cmp(NearCmpView v, int64_t obase, const double2 *x, double2 *part)
{
    __shared__ double2 sxr[kCmpRows];
    __shared__ double2 syc[3][256];
    // issue priority of these waves over others resident on the same SIMD (the
    // coupling kernel runs beside this one); a compile-time choice, so the kernel's
    // registers are those of the plain form
    near_cmp_item<U, RS, PRIO>(v, v.order[obase + blockIdx.x], x, part, sxr, syc);
}

// Both kinds of work items in one launch: the nw wide ones first (launch order
// positions na .. na + nw - 1, UW column groups per lane), then the na narrow ones
// (two column groups); one launch tail instead of two
// (at most 96 registers, five waves per SIMD: alone 73 against 76 us at 102)
template <int UW, int PRIO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_near_cmp1(
    NearCmpView v, int64_t na, int64_t nw, const double2 *x, double2 *part)
{
    __shared__ double2 sxr[kCmpRows];
    __shared__ double2 syc[3][256];
    const int64_t b = blockIdx.x;
    if (b < nw) near_cmp_item<UW, 2, PRIO>(v, v.order[na + b], x, part, sxr, syc);
    else near_cmp_item<2, 2, PRIO>(v, v.order[b - nw], x, part, sxr, syc);
}

// Values of the once-per-entry near field: entry (i, j) is the sum over the leaf
// slots holding i and those holding j (ascending) of the leaf-pair block entries,
// (B_ts)[slot_t(i)][slot_s(j)] for t <= s and (B_st)[slot_s(j)][slot_t(i)] for t > s,
// for the near leaf pairs only.
__global__ __launch_bounds__(256) void k_near_merge(NearCmpView v, const double2 *bval, int nF)
{
    const int64_t k = blockIdx.x;
    const int nr = v.nr[k], nc = v.nc[k], ld = v.ld[k];
    const int32_t *rows = v.idx + v.lst[k], *cols = rows + nr;
    double2 *out = v.val + v.val_off[k];
    for (int64_t e = threadIdx.x; e < (int64_t)nr * ld; e += blockDim.x) {
        const int kr = (int)(e / ld), kc = (int)(e % ld);
        if (kc >= nc) {   // row padding
            out[e] = make_double2(0.0, 0.0);
            continue;
        }
        const int32_t i = rows[kr], j = cols[kc];
        double re = 0.0, im = 0.0;
        for (int a = v.occ_ptr[i]; a < v.occ_ptr[i + 1]; ++a) {
            const int32_t qa = v.occ[a];
            const int t = qa / nF, st = qa % nF;
            const int p0 = v.np_ptr[t], p1 = v.np_ptr[t + 1];
            for (int b = v.occ_ptr[j]; b < v.occ_ptr[j + 1]; ++b) {
                const int32_t qb = v.occ[b];
                const int sl = qb / nF, ss = qb % nF;
                int lo = p0, hi = p1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (v.np_leaf[mid] < sl) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < p1 && v.np_leaf[lo] == sl) {
                    const int code = v.np_code[lo];
                    const int64_t blk = code >> 1;
                    const double2 val = (code & 1) ? bval[((size_t)blk * nF + ss) * nF + st]
                                                   : bval[((size_t)blk * nF + st) * nF + ss];
                    re += val.x;
                    im += val.y;
                }
            }
        }
        out[e] = make_double2(re, im);
    }
}

}  // namespace

int near_cmp_max() { return 256; }

void launch_near_merge(ige_op op)
{
    const NearCmpView &v = op->cview;
    if (!op->cmp_on || v.nsub == 0) return;
    hipLaunchKernelGGL(k_near_merge, dim3((unsigned)v.nsub), dim3(256), 0, lstream(op), v, op->view.bval, op->view.nF);
    IGE_HIP(hipGetLastError());
}

void launch_near_once(ige_op op, const double2 *x, double2 *part, hipStream_t st)
{
    const NearCmpView &v = op->cview;
    const dim3 blk(256);
    const int64_t na = op->cmp.nnarrow, nw = v.nwork - na;
    const bool pr = op->near_prio > 0;
    if (op->near_one && op->cmp_rs == 2 && (op->cmp.maxn + 63) / 64 <= 3 && na + nw > 0) {
        const dim3 grid((unsigned)(na + nw));
        if (pr) hipLaunchKernelGGL((k_near_cmp1<3, 1>), grid, blk, 0, st, v, na, nw, x, part);
        else hipLaunchKernelGGL((k_near_cmp1<3, 0>), grid, blk, 0, st, v, na, nw, x, part);
        IGE_HIP(hipGetLastError());
        return;
    }
    if (na > 0) {
        const dim3 grid((unsigned)na);
        if (op->cmp_rs == 4) {
            if (pr) hipLaunchKernelGGL((k_near_cmp<2, 4, 1>), grid, blk, 0, st, v, (int64_t)0, x, part);
            else hipLaunchKernelGGL((k_near_cmp<2, 4, 0>), grid, blk, 0, st, v, (int64_t)0, x, part);
        } else {
            if (pr) hipLaunchKernelGGL((k_near_cmp<2, 2, 1>), grid, blk, 0, st, v, (int64_t)0, x, part);
            else hipLaunchKernelGGL((k_near_cmp<2, 2, 0>), grid, blk, 0, st, v, (int64_t)0, x, part);
        }
        IGE_HIP(hipGetLastError());
    }
    if (nw > 0) {
        const dim3 grid((unsigned)nw);
        if ((op->cmp.maxn + 63) / 64 <= 3) {
            if (pr) hipLaunchKernelGGL((k_near_cmp<3, 2, 1>), grid, blk, 0, st, v, na, x, part);
            else hipLaunchKernelGGL((k_near_cmp<3, 2, 0>), grid, blk, 0, st, v, na, x, part);
        } else {
            if (pr) hipLaunchKernelGGL((k_near_cmp<4, 2, 1>), grid, blk, 0, st, v, na, x, part);
            else hipLaunchKernelGGL((k_near_cmp<4, 2, 0>), grid, blk, 0, st, v, na, x, part);
        }
        IGE_HIP(hipGetLastError());
    }
}

}  // namespace ige
