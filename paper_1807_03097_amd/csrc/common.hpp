// Shared definitions of the igaefie library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/igaefie.h"

namespace ige {

constexpr int kMaxGeomDeg = 8;   // NURBS degree of the input patches
constexpr int kMaxP = 4;         // discretisation degree p
constexpr int kMaxNl = 2 * kMaxP * (kMaxP + 1);   // local glued functions per element
constexpr int kMaxQ1 = 16;       // q + 1
constexpr int kMaxLev = 11;      // cluster-tree levels 0..10
constexpr int kMaxG = 8;         // regular Gauss points per direction
constexpr int kMaxGs = 12;       // singular sub-rule points per variable

// ---------------------------------------------------------------------------
// rational Bezier form of the patches (one rational Bezier patch per knot span)
// ---------------------------------------------------------------------------
struct PatchHdr {
    int pu, pv;       // degrees
    int su, sv;       // spans per direction
    int brk_u, brk_v; // offsets of the span breakpoints (su+1, sv+1 values) in brk[]
    int cp;           // offset of the homogeneous control points in cp[]:
                      // [span_v][span_u][j2 <= pv][j1 <= pu][4] = (w x, w y, w z, w)
};

struct GeomView {
    const PatchHdr *hdr;
    const double *brk;
    const double *cp;
};

// Evaluate F, d_uF, d_vF of patch j at parameter (u, v) from the Bezier form.
__host__ __device__ inline void bezier_eval(const GeomView &g, int j, double u, double v, double X[3], double Xu[3],
                                            double Xv[3])
{
    const PatchHdr h = g.hdr[j];
    int su = 0, sv = 0;
    while (su < h.su - 1 && u >= g.brk[h.brk_u + su + 1]) ++su;
    while (sv < h.sv - 1 && v >= g.brk[h.brk_v + sv + 1]) ++sv;
    const double ua = g.brk[h.brk_u + su], ub = g.brk[h.brk_u + su + 1];
    const double va = g.brk[h.brk_v + sv], vb = g.brk[h.brk_v + sv + 1];
    const double t = (u - ua) / (ub - ua), s = (v - va) / (vb - va);
    // Bernstein values and derivatives (w.r.t. the span-local variable)
    double Bu[kMaxGeomDeg + 1], Du[kMaxGeomDeg + 1], Bv[kMaxGeomDeg + 1], Dv[kMaxGeomDeg + 1];
    auto bern = [](int p, double x, double *B, double *D) {
        // degree p-1 values first (for derivatives), built by the de Casteljau-type
        // triangle B_i^k = (1-x) B_i^{k-1} + x B_{i-1}^{k-1}
        double T[kMaxGeomDeg + 1];
        T[0] = 1.0;
        for (int k = 1; k < p; ++k) {
            T[k] = x * T[k - 1];
            for (int i = k - 1; i >= 1; --i) T[i] = (1.0 - x) * T[i] + x * T[i - 1];
            T[0] = (1.0 - x) * T[0];
        }
        // T holds degree p-1 (if p >= 1)
        for (int i = 0; i <= p; ++i) {
            double lo = (i >= 1) ? T[i - 1] : 0.0;
            double hi = (i <= p - 1) ? T[i] : 0.0;
            D[i] = p * (lo - hi);
            B[i] = (1.0 - x) * hi + x * lo;
        }
        if (p == 0) { B[0] = 1.0; D[0] = 0.0; }
    };
    bern(h.pu, t, Bu, Du);
    bern(h.pv, s, Bv, Dv);
    const double *c = g.cp + h.cp + (size_t)(sv * h.su + su) * (h.pv + 1) * (h.pu + 1) * 4;
    double A[4] = {0, 0, 0, 0}, Au[4] = {0, 0, 0, 0}, Av[4] = {0, 0, 0, 0};
    for (int j2 = 0; j2 <= h.pv; ++j2)
        for (int j1 = 0; j1 <= h.pu; ++j1) {
            const double *P = c + (j2 * (h.pu + 1) + j1) * 4;
            const double b = Bu[j1] * Bv[j2], bu = Du[j1] * Bv[j2], bv = Bu[j1] * Dv[j2];
            for (int k = 0; k < 4; ++k) {
                A[k] += b * P[k];
                Au[k] += bu * P[k];
                Av[k] += bv * P[k];
            }
        }
    const double iw = 1.0 / A[3], du = 1.0 / (ub - ua), dv = 1.0 / (vb - va);
    for (int k = 0; k < 3; ++k) {
        X[k] = A[k] * iw;
        Xu[k] = (Au[k] - X[k] * Au[3]) * iw * du;
        Xv[k] = (Av[k] - X[k] * Av[3]) * iw * dv;
    }
}

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

struct Status {
    int code;
    std::string msg;
};

#define IGE_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            throw ::ige::Status{IGE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
        }                                                                                   \
    } while (0)

#define IGE_REQUIRE(cond, msg)                                     \
    do {                                                           \
        if (!(cond)) throw ::ige::Status{IGE_EINVAL, (msg)};       \
    } while (0)

// device buffer owned by the operator
template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    void alloc(size_t count)
    {
        release();
        n = count;
        if (count) {
            hipError_t e = hipMalloc((void **)&p, sizeof(T) * count);
            if (e != hipSuccess) {
                p = nullptr;
                n = 0;
                throw Status{IGE_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed"};
            }
        }
    }
    void upload(const std::vector<T> &v, hipStream_t s)
    {
        alloc(v.size());
        if (!v.empty()) IGE_HIP(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return sizeof(T) * n; }
    ~DBuf() { release(); }
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
};

// pinned host buffer (for small device-to-host transfers inside iterations)
template <typename T>
struct HBuf {
    T *p = nullptr;
    size_t n = 0;
    void ensure(size_t count)
    {
        if (count <= n) return;
        release();
        if (hipHostMalloc((void **)&p, sizeof(T) * count, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            throw Status{IGE_ENOMEM, "hipHostMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed"};
        }
        n = count;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    ~HBuf() { release(); }
    HBuf() = default;
    HBuf(const HBuf &) = delete;
    HBuf &operator=(const HBuf &) = delete;
};

}  // namespace ige
