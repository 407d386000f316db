// Host-side set-up of the igaefie operator (see setup.hpp).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>

namespace ige {

// ---------------------------------------------------------------------------
// Gauss-Legendre nodes on [0,1] (Newton on P_n with the derivative identity
// (1-x^2) P_n' = n (P_{n-1} - x P_n)), Chebyshev nodes and barycentric Lagrange
// ---------------------------------------------------------------------------
void gauss_legendre01(int n, double *x, double *w)
{
    const int half = (n + 1) / 2;
    for (int i = 0; i < half; ++i) {
        // Tricomi-type initial guess for the i-th largest root
        double z = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double pn = 0.0, pn1 = 0.0;
        for (int it = 0; it < 60; ++it) {
            double a = 1.0, b = z;   // P_0, P_1
            if (n == 1) { pn = z; pn1 = 1.0; }
            for (int k = 2; k <= n; ++k) {
                double c = ((2.0 * k - 1.0) * z * b - (k - 1.0) * a) / k;
                a = b;
                b = c;
            }
            if (n > 1) { pn = b; pn1 = a; }
            double dp = n * (pn1 - z * pn) / (1.0 - z * z);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-17) break;
        }
        double a = 1.0, b = z;
        for (int k = 2; k <= n; ++k) {
            double c = ((2.0 * k - 1.0) * z * b - (k - 1.0) * a) / k;
            a = b;
            b = c;
        }
        if (n == 1) { b = z; a = 1.0; }
        double dp = n * (a - z * b) / (1.0 - z * z);
        double wi = 1.0 / ((1.0 - z * z) * dp * dp);   // half of the [-1,1] weight
        x[n - 1 - i] = 0.5 + 0.5 * z;
        w[n - 1 - i] = wi;
        x[i] = 0.5 - 0.5 * z;
        w[i] = wi;
    }
}

void chebyshev01(int q, double *x)
{
    for (int m = 0; m <= q; ++m) x[m] = 0.5 + 0.5 * std::cos(M_PI * (2.0 * m + 1.0) / (2.0 * q + 2.0));
}

void lagrange_bary(int q, const double *xn, double s, double *L)
{
    // barycentric weights
    double wb[kMaxQ1];
    for (int m = 0; m <= q; ++m) {
        double prod = 1.0;
        for (int k = 0; k <= q; ++k)
            if (k != m) prod *= (xn[m] - xn[k]);
        wb[m] = 1.0 / prod;
    }
    for (int m = 0; m <= q; ++m)
        if (s == xn[m]) {
            for (int k = 0; k <= q; ++k) L[k] = (k == m) ? 1.0 : 0.0;
            return;
        }
    double l = 1.0;
    for (int k = 0; k <= q; ++k) l *= (s - xn[k]);
    for (int m = 0; m <= q; ++m) L[m] = l * wb[m] / (s - xn[m]);
}

// ---------------------------------------------------------------------------
// geometry: validation, Bezier extraction by knot insertion, edge matching
// ---------------------------------------------------------------------------
namespace {

using H4 = std::array<double, 4>;

// Insert knot t once (Boehm), homogeneous points.
void insert_knot(std::vector<double> &U, int p, std::vector<H4> &Pt, double t)
{
    const int npt = (int)Pt.size();
    int k = -1;
    for (int i = 0; i + 1 < (int)U.size(); ++i)
        if (U[i] <= t && t < U[i + 1]) k = i;
    std::vector<H4> Q(npt + 1);
    for (int i = 0; i <= npt; ++i) {
        if (i <= k - p) {
            Q[i] = Pt[i];
        } else if (i >= k + 1) {
            Q[i] = Pt[i - 1];
        } else {
            const double a = (t - U[i]) / (U[i + p] - U[i]);
            for (int c = 0; c < 4; ++c) Q[i][c] = a * Pt[i][c] + (1.0 - a) * Pt[i - 1][c];
        }
    }
    U.insert(U.begin() + k + 1, t);
    Pt.swap(Q);
}

// Raise every interior knot to multiplicity p: the control points then group into
// rational Bezier segments of p+1 points sharing end points.
void extract_1d(std::vector<double> U, int p, std::vector<H4> &Pt, std::vector<double> &brk)
{
    std::vector<double> interior;
    for (size_t i = p + 1; i + p + 1 < U.size(); ++i) interior.push_back(U[i]);
    std::map<double, int> mult;
    for (double t : interior) mult[t]++;
    for (auto &kv : mult)
        for (int r = kv.second; r < p; ++r) insert_knot(U, p, Pt, kv.first);
    brk.clear();
    brk.push_back(0.0);
    for (auto &kv : mult) brk.push_back(kv.first);
    brk.push_back(1.0);
}

double dist3(const double *a, const double *b)
{
    return std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
}

// parameter point of patch edge k at edge parameter t (0: v=0, 1: u=1, 2: v=1, 3: u=0)
void edge_uv(int k, double t, double &u, double &v)
{
    switch (k) {
        case 0: u = t; v = 0.0; break;
        case 1: u = 1.0; v = t; break;
        case 2: u = t; v = 1.0; break;
        default: u = 0.0; v = t; break;
    }
}

}  // namespace

void build_geometry(Geometry &G, int P, const int *degree, const int *n_ctrl, const double *knots,
                    const double *ctrl)
{
    IGE_REQUIRE(P >= 1 && P <= (1 << 20), "n_patches must be positive");
    IGE_REQUIRE(degree && n_ctrl && knots && ctrl, "null geometry pointer");
    G.P = P;
    G.hdr.assign(P, PatchHdr{});
    G.brk.clear();
    G.cp.clear();
    size_t ko = 0, co = 0;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int j = 0; j < P; ++j) {
        const int pu = degree[2 * j], pv = degree[2 * j + 1], nu = n_ctrl[2 * j], nv = n_ctrl[2 * j + 1];
        IGE_REQUIRE(pu >= 1 && pu <= kMaxGeomDeg && pv >= 1 && pv <= kMaxGeomDeg, "patch degree must be 1..8");
        IGE_REQUIRE(nu >= pu + 1 && nv >= pv + 1 && nu <= 4096 && nv <= 4096, "too few control points for degree");
        std::vector<double> U(knots + ko, knots + ko + nu + pu + 1);
        ko += nu + pu + 1;
        std::vector<double> V(knots + ko, knots + ko + nv + pv + 1);
        ko += nv + pv + 1;
        for (auto *K : {&U, &V}) {
            const int pp = (K == &U) ? pu : pv;
            for (size_t i = 0; i + 1 < K->size(); ++i)
                IGE_REQUIRE(std::isfinite((*K)[i]) && (*K)[i] <= (*K)[i + 1], "knot vector must be non-decreasing");
            for (int i = 0; i <= pp; ++i)
                IGE_REQUIRE((*K)[i] == 0.0 && (*K)[K->size() - 1 - i] == 1.0, "knot vectors must be open on [0,1]");
            std::map<double, int> mult;
            for (size_t i = pp + 1; i + pp + 1 < K->size(); ++i) mult[(*K)[i]]++;
            for (auto &kv : mult) IGE_REQUIRE(kv.second <= pp, "interior knot multiplicity exceeds the degree");
        }
        // homogeneous control net [nv][nu]
        std::vector<std::vector<H4>> rows(nv, std::vector<H4>(nu));
        for (int j2 = 0; j2 < nv; ++j2)
            for (int j1 = 0; j1 < nu; ++j1) {
                const double *c = ctrl + (co + (size_t)j2 * nu + j1) * 4;
                IGE_REQUIRE(std::isfinite(c[0]) && std::isfinite(c[1]) && std::isfinite(c[2]) && std::isfinite(c[3]) &&
                                c[3] > 0.0,
                            "control points must be finite with positive weights");
                rows[j2][j1] = {c[0] * c[3], c[1] * c[3], c[2] * c[3], c[3]};
                for (int k = 0; k < 3; ++k) {
                    lo[k] = std::min(lo[k], c[k]);
                    hi[k] = std::max(hi[k], c[k]);
                }
            }
        co += (size_t)nu * nv;
        // extract along u for every row, then along v for every column
        std::vector<double> bu, bv;
        for (int j2 = 0; j2 < nv; ++j2) extract_1d(U, pu, rows[j2], bu);
        const int nu2 = (int)rows[0].size();
        std::vector<std::vector<H4>> cols(nu2, std::vector<H4>(nv));
        for (int j1 = 0; j1 < nu2; ++j1) {
            for (int j2 = 0; j2 < nv; ++j2) cols[j1][j2] = rows[j2][j1];
            extract_1d(V, pv, cols[j1], bv);
        }
        const int nv2 = (int)cols[0].size();
        const int su = (int)bu.size() - 1, sv = (int)bv.size() - 1;
        IGE_REQUIRE(nu2 == su * pu + 1 && nv2 == sv * pv + 1, "Bezier extraction size mismatch");
        PatchHdr &h = G.hdr[j];
        h.pu = pu; h.pv = pv; h.su = su; h.sv = sv;
        h.brk_u = (int)G.brk.size();
        G.brk.insert(G.brk.end(), bu.begin(), bu.end());
        h.brk_v = (int)G.brk.size();
        G.brk.insert(G.brk.end(), bv.begin(), bv.end());
        h.cp = (int)G.cp.size();
        for (int s2 = 0; s2 < sv; ++s2)
            for (int s1 = 0; s1 < su; ++s1)
                for (int j2 = 0; j2 <= pv; ++j2)
                    for (int j1 = 0; j1 <= pu; ++j1) {
                        const H4 &c = cols[s1 * pu + j1][s2 * pv + j2];
                        G.cp.insert(G.cp.end(), c.begin(), c.end());
                    }
    }
    G.scale = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    IGE_REQUIRE(G.scale > 0.0, "degenerate geometry");

    // edge matching: endpoints and midpoint coincide (forward or reversed); the
    // quarter points must coincide too (interfaces coincide as parametrised curves)
    const GeomView gv = G.view();
    const double tol = 1e-9 * G.scale;
    const double ts[5] = {0.0, 0.25, 0.5, 0.75, 1.0};
    std::vector<double> E((size_t)P * 4 * 5 * 3);
    for (int j = 0; j < P; ++j)
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 5; ++i) {
                double u, v, Xu[3], Xv[3];
                edge_uv(k, ts[i], u, v);
                bezier_eval(gv, j, u, v, &E[(((size_t)j * 4 + k) * 5 + i) * 3], Xu, Xv);
            }
    auto pt = [&](int j, int k, int i) { return &E[(((size_t)j * 4 + k) * 5 + i) * 3]; };
    G.partner.assign((size_t)P * 4, {-1, -1, 0});
    for (int a = 0; a < P * 4; ++a) {
        int found = 0;
        for (int b = 0; b < P * 4; ++b) {
            if (a == b) continue;
            const int ja = a / 4, ka = a % 4, jb = b / 4, kb = b % 4;
            bool fwd = dist3(pt(ja, ka, 0), pt(jb, kb, 0)) <= tol && dist3(pt(ja, ka, 4), pt(jb, kb, 4)) <= tol &&
                       dist3(pt(ja, ka, 2), pt(jb, kb, 2)) <= tol;
            bool rev = dist3(pt(ja, ka, 0), pt(jb, kb, 4)) <= tol && dist3(pt(ja, ka, 4), pt(jb, kb, 0)) <= tol &&
                       dist3(pt(ja, ka, 2), pt(jb, kb, 2)) <= tol;
            if (!fwd && !rev) continue;
            for (int i = 0; i < 5; ++i) {
                const double *q = pt(jb, kb, rev ? 4 - i : i);
                IGE_REQUIRE(dist3(pt(ja, ka, i), q) <= tol,
                            "patch interface " + std::to_string(ja) + "/" + std::to_string(jb) +
                                " does not coincide as a parametrised curve");
            }
            G.partner[a] = {jb, kb, rev ? 1 : 0};
            ++found;
        }
        IGE_REQUIRE(found == 1, "patch " + std::to_string(a / 4) + " edge " + std::to_string(a % 4) + " has " +
                                    std::to_string(found) + " partner edges; a closed conforming surface is required");
    }
}

// ---------------------------------------------------------------------------
// discretisation: canonical glued unknowns and 1-D Bezier extraction
// ---------------------------------------------------------------------------
namespace {

// The p+1 B-splines of degree p that are nonzero on knot span `span` of U, as the
// polynomial piece of that span (triangular scheme with left/right differences).
void basis_piece(const std::vector<double> &U, int span, int p, double x, double *N)
{
    double left[kMaxP + 2], right[kMaxP + 2];
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - U[span + 1 - j];
        right[j] = U[span + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            const double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}

double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// solve the small dense system A c = b (partial pivoting), A row-major n x n
void small_solve(int n, std::vector<double> A, double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int k = c + 1; k < n; ++k) b[c] -= A[c * n + k] * b[k];
        b[c] /= A[c * n + c];
    }
}

// Bernstein coefficients of the degree-`deg` pieces of the uniform open splines on
// each of the n elements, by interpolation at deg+1 equispaced element points.
void extraction_1d(int deg, int n, std::vector<double> &ext)
{
    const int k1 = deg + 1;
    ext.assign((size_t)n * k1 * k1, 0.0);
    if (deg == 0) {
        for (int e = 0; e < n; ++e) ext[e] = 1.0;
        return;
    }
    std::vector<double> U;
    for (int i = 0; i <= deg; ++i) U.push_back(0.0);
    for (int i = 1; i < n; ++i) U.push_back((double)i / n);
    for (int i = 0; i <= deg; ++i) U.push_back(1.0);
    std::vector<double> V((size_t)k1 * k1);
    for (int r = 0; r < k1; ++r) {
        const double s = (double)r / deg;
        for (int a = 0; a < k1; ++a) V[r * k1 + a] = binom(deg, a) * std::pow(s, a) * std::pow(1.0 - s, deg - a);
    }
    for (int e = 0; e < n; ++e) {
        double vals[kMaxP + 2][kMaxP + 2];   // vals[r][t]
        for (int r = 0; r < k1; ++r) {
            const double u = (e + (double)r / deg) / n;
            basis_piece(U, e + deg, deg, u, vals[r]);
        }
        for (int t = 0; t < k1; ++t) {
            double b[kMaxP + 2];
            for (int r = 0; r < k1; ++r) b[r] = vals[r][t];
            small_solve(k1, V, b);
            for (int a = 0; a < k1; ++a) ext[((size_t)e * k1 + t) * k1 + a] = b[a];
        }
    }
}

}  // namespace

void build_discretisation(Discretisation &D, const Geometry &G, int p, int m, int scalar)
{
    IGE_REQUIRE(p >= 1 && p <= kMaxP, "p must be 1..4");
    IGE_REQUIRE(m >= 0 && m <= 10, "level must be 0..10");
    D.P = G.P; D.p = p; D.m = m; D.n = 1 << m; D.nb = D.n + p;
    D.scalar = scalar;
    const int n = D.n, nb = D.nb;
    D.dof.assign((size_t)D.P * 2 * nb * nb, -1);
    D.sgn.assign((size_t)D.P * 2 * nb * nb, 0);
    auto at = [&](int j, int a, int i2, int i1) { return (((size_t)j * 2 + a) * nb + i2) * nb + i1; };
    if (scalar) {
        // scalar single layer: the (n+p)^2 tensor B-splines of degree p of every patch,
        // numbered patch, i2, i1, in slot 0 of the table (the density space needs no
        // continuity across patches)
        int N = 0;
        D.inc.clear();
        for (int j = 0; j < D.P; ++j)
            for (int i2 = 0; i2 < nb; ++i2)
                for (int i1 = 0; i1 < nb; ++i1) {
                    D.dof[at(j, 0, i2, i1)] = N++;
                    D.sgn[at(j, 0, i2, i1)] = 1;
                    D.inc.push_back({j, 0, i1, i2, 1});
                    D.inc.push_back({-1, 0, 0, 0, 0});
                }
        D.N = N;
        extraction_1d(p, n, D.ext_p);
        extraction_1d(p - 1, n, D.ext_q);
        return;
    }
    // outward conormal side of each edge: -1 for u=0 / v=0, +1 for u=1 / v=1
    const int side[4] = {-1, +1, +1, -1};
    int N = 0;
    for (int j = 0; j < D.P; ++j)
        for (int a = 0; a < 2; ++a) {
            const int r1 = (a == 0) ? n + p : n + p - 1, r2 = (a == 0) ? n + p - 1 : n + p;
            for (int i2 = 0; i2 < r2; ++i2)
                for (int i1 = 0; i1 < r1; ++i1) {
                    if (D.dof[at(j, a, i2, i1)] >= 0) continue;
                    D.dof[at(j, a, i2, i1)] = N;
                    D.sgn[at(j, a, i2, i1)] = 1;
                    // normal-flux unknown on a patch edge?
                    int edge = -1, tpos = 0;
                    if (a == 0 && i1 == 0) { edge = 3; tpos = i2; }
                    else if (a == 0 && i1 == n + p - 1) { edge = 1; tpos = i2; }
                    else if (a == 1 && i2 == 0) { edge = 0; tpos = i1; }
                    else if (a == 1 && i2 == n + p - 1) { edge = 2; tpos = i1; }
                    if (edge >= 0) {
                        const auto pr = G.partner[(size_t)j * 4 + edge];
                        const int jb = pr[0], kb = pr[1];
                        const int tb = pr[2] ? (n + p - 2 - tpos) : tpos;
                        int ab, b1, b2;
                        switch (kb) {
                            case 0: ab = 1; b1 = tb; b2 = 0; break;
                            case 1: ab = 0; b1 = n + p - 1; b2 = tb; break;
                            case 2: ab = 1; b1 = tb; b2 = n + p - 1; break;
                            default: ab = 0; b1 = 0; b2 = tb; break;
                        }
                        IGE_REQUIRE(D.dof[at(jb, ab, b2, b1)] < 0, "interface unknown matched twice");
                        D.dof[at(jb, ab, b2, b1)] = N;
                        D.sgn[at(jb, ab, b2, b1)] = (int8_t)(-side[edge] * side[kb]);
                    }
                    ++N;
                }
        }
    D.N = N;
    D.inc.assign((size_t)N * 2, {-1, 0, 0, 0, 0});
    for (int j = 0; j < D.P; ++j)
        for (int a = 0; a < 2; ++a)
            for (int i2 = 0; i2 < nb; ++i2)
                for (int i1 = 0; i1 < nb; ++i1) {
                    const int32_t d = D.dof[at(j, a, i2, i1)];
                    if (d < 0) continue;
                    auto &slot = (D.inc[(size_t)d * 2][0] < 0) ? D.inc[(size_t)d * 2] : D.inc[(size_t)d * 2 + 1];
                    slot = {j, a, i1, i2, D.sgn[at(j, a, i2, i1)]};
                }
    extraction_1d(p, n, D.ext_p);
    extraction_1d(p - 1, n, D.ext_q);
}

// ---------------------------------------------------------------------------
// cluster tree, bounding balls, Algorithm 1
// ---------------------------------------------------------------------------
namespace {

struct Balls {
    std::vector<double> c;   // [ncl][3]
    std::vector<double> r;
};

// element vertex images, [P][n+1][n+1][3]
std::vector<double> vertex_images(const Geometry &G, int n)
{
    const GeomView gv = G.view();
    std::vector<double> V((size_t)G.P * (n + 1) * (n + 1) * 3);
    for (int j = 0; j < G.P; ++j)
        for (int b = 0; b <= n; ++b)
            for (int a = 0; a <= n; ++a) {
                double Xu[3], Xv[3];
                bezier_eval(gv, j, (double)a / n, (double)b / n, &V[(((size_t)j * (n + 1) + b) * (n + 1) + a) * 3], Xu,
                            Xv);
            }
    return V;
}

Balls level_balls(const Geometry &G, int n, int lvl, const std::vector<double> &V)
{
    const GeomView gv = G.view();
    const int s = 1 << lvl, sub = n / s;
    Balls B;
    B.c.resize((size_t)G.P * s * s * 3);
    B.r.resize((size_t)G.P * s * s);
    for (int j = 0; j < G.P; ++j)
        for (int k2 = 0; k2 < s; ++k2)
            for (int k1 = 0; k1 < s; ++k1) {
                const size_t id = ((size_t)j * s + k2) * s + k1;
                double *c = &B.c[id * 3], Xu[3], Xv[3];
                bezier_eval(gv, j, (k1 + 0.5) / s, (k2 + 0.5) / s, c, Xu, Xv);
                double r = 0.0;
                for (int b = k2 * sub; b <= (k2 + 1) * sub; ++b)
                    for (int a = k1 * sub; a <= (k1 + 1) * sub; ++a)
                        r = std::max(r, dist3(c, &V[(((size_t)j * (n + 1) + b) * (n + 1) + a) * 3]));
                B.r[id] = r;
            }
    return B;
}

}  // namespace

void build_partition(Partition &T, const Geometry &G, const Discretisation &D, double eta, int leaf_depth, double kappa,
                     double kappa_cap)
{
    const int n = D.n;
    T.L = std::max(0, D.m - leaf_depth);
    T.s = n >> T.L;
    T.far.clear();
    T.near.clear();
    const std::vector<double> V = vertex_images(G, n);
    // admissible iff max diam <= eta * dist * (1 - 1e-9): the relative margin keeps
    // the decision independent of rounding when the two sides tie exactly
    const double margin = 1.0 - 1e-9;
    std::vector<std::pair<int32_t, int32_t>> cand;
    for (int a = 0; a < G.P; ++a)
        for (int b = 0; b < G.P; ++b) cand.push_back({a, b});
    T.diam.assign((size_t)T.L + 1, 0.0);
    for (int l = 0; l <= T.L; ++l) {
        const Balls B = level_balls(G, n, l, V);
        for (double r : B.r) T.diam[l] = std::max(T.diam[l], 2.0 * r);
        const int s = 1 << l;
        std::vector<std::pair<int32_t, int32_t>> next;
        for (auto &pr : cand) {
            const int t = pr.first, u = pr.second;
            const double dist = dist3(&B.c[(size_t)t * 3], &B.c[(size_t)u * 3]) - B.r[t] - B.r[u];
            const double diam = 2.0 * std::max(B.r[t], B.r[u]);
            // optional wavenumber cap: admissible only if also kappa * diam <= kappa_cap
            const bool adm = eta > 0.0 && dist > 0.0 && diam <= eta * dist * margin &&
                             (kappa_cap <= 0.0 || kappa * diam <= kappa_cap * margin);
            if (adm) {
                T.far.push_back({l, t, u});
            } else if (l == T.L) {
                T.near.push_back({t, u});
            } else {
                auto kids = [&](int cid, int out[4]) {
                    const int j = cid / (s * s), r = cid % (s * s), k2 = r / s, k1 = r % s;
                    int i = 0;
                    for (int c2 = 0; c2 < 2; ++c2)
                        for (int c1 = 0; c1 < 2; ++c1) out[i++] = (j * 2 * s + 2 * k2 + c2) * 2 * s + 2 * k1 + c1;
                };
                int kt[4], ku[4];
                kids(t, kt);
                kids(u, ku);
                for (int x = 0; x < 4; ++x)
                    for (int y = 0; y < 4; ++y) next.push_back({kt[x], ku[y]});
            }
        }
        cand.swap(next);
        if (l == T.L) break;
    }
    std::sort(T.far.begin(), T.far.end());
    std::sort(T.near.begin(), T.near.end());
}

// ---------------------------------------------------------------------------
// near-field sparsity pattern in the glued basis
// ---------------------------------------------------------------------------
void build_near_blocks(NearBlocks &B, const Discretisation &D, const Partition &T, int nch)
{
    const int p = D.p, nb = D.nb, s = T.s, S = 1 << T.L;
    const int W = s + p;
    B.W = W;
    // slots: EFIE W (W-1) per flux component; scalar W x W functions (slot i2 W + i1)
    B.nF = D.scalar ? W * W : 2 * W * (W - 1);
    IGE_REQUIRE(B.nF <= kMaxLeafSlots, "leaf clusters too large for the near-field blocks (lower leaf_depth)");
    const int nF = B.nF;
    const size_t nleaf = (size_t)D.P * S * S;
    B.leafdof.assign(nleaf * nF, -1);
    B.leafsgn.assign(nleaf * nF, 0);
    for (int j = 0; j < D.P; ++j)
        for (int k2 = 0; k2 < S; ++k2)
            for (int k1 = 0; k1 < S; ++k1) {
                const size_t lid = ((size_t)j * S + k2) * S + k1;
                for (int a = 0; a < (D.scalar ? 1 : 2); ++a) {
                    const int w1 = (a == 0) ? W : W - 1, w2 = (a == 0 && !D.scalar) ? W - 1 : W;
                    for (int i2 = 0; i2 < w2; ++i2)
                        for (int i1 = 0; i1 < w1; ++i1) {
                            const size_t off = (((size_t)j * 2 + a) * nb + k2 * s + i2) * nb + k1 * s + i1;
                            const int k = leaf_slot(W, a, i1, i2);
                            B.leafdof[lid * nF + k] = D.dof[off];
                            B.leafsgn[lid * nF + k] = D.dof[off] >= 0 ? D.sgn[off] : 0;
                        }
                }
            }
    // one block per unordered pair; the block tree is symmetric
    B.pair.clear();
    for (const auto &np : T.near) {
        if (np[0] > np[1]) continue;
        IGE_REQUIRE(std::binary_search(T.near.begin(), T.near.end(), std::array<int32_t, 2>{np[1], np[0]}),
                    "near leaf pairs are not symmetric");
        B.pair.push_back(np[0]);
        B.pair.push_back(np[1]);
    }
    B.nch = std::max(1, std::min(nch, nF));
    B.rc = (nF + B.nch - 1) / B.nch;
    B.nch = (nF + B.rc - 1) / B.rc;
    const int64_t nblk = B.nblk();
    IGE_REQUIRE(B.nslots() < ((int64_t)1 << 31), "near field too large for 32-bit partial indices");
    // fixed-order reduction lists: for every unknown its row partials and (for
    // off-diagonal blocks) its column partials, in block order
    std::vector<int64_t> cnt((size_t)D.N + 1, 0);
    auto visit = [&](auto &&emit) {
        for (int64_t b = 0; b < nblk; ++b) {
            const int lt = B.pair[2 * b], ls = B.pair[2 * b + 1];
            for (int k = 0; k < nF; ++k) {
                const int32_t d = B.leafdof[(size_t)lt * nF + k];
                if (d >= 0) emit(d, b * nF + k);
            }
            if (lt == ls) continue;
            for (int ch = 0; ch < B.nch; ++ch)
                for (int k = 0; k < nF; ++k) {
                    const int32_t d = B.leafdof[(size_t)ls * nF + k];
                    if (d >= 0) emit(d, nblk * nF + (b * B.nch + ch) * nF + k);
                }
        }
    };
    visit([&](int32_t d, int64_t) { cnt[d + 1]++; });
    for (int i = 0; i < D.N; ++i) cnt[i + 1] += cnt[i];
    B.red_ptr = cnt;
    B.red_idx.assign(cnt[D.N], 0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    visit([&](int32_t d, int64_t slot) { B.red_idx[fill[d]++] = (int32_t)slot; });
}

// ---------------------------------------------------------------------------
// near field stored once per distinct entry (owner blocks split into dense rectangles)
// ---------------------------------------------------------------------------
void build_near_compact(NearCompact &C, const Discretisation &D, const Partition &T, const NearBlocks &B,
                        int rows_per_item)
{
    C = NearCompact{};
    const int p = D.p, n = D.n, nb = D.nb, s = T.s, SL = 1 << T.L, nF = B.nF;
    const int nleaf = D.P * SL * SL;
    const int64_t N = D.N;
    // owner leaf of every unknown: leaf of the last element of its support at its first
    // incarnation in canonical order
    std::vector<int32_t> own((size_t)N, -1);
    for (int j = 0; j < D.P; ++j)
        for (int a = 0; a < (D.scalar ? 1 : 2); ++a) {
            const int n1 = a == 0 ? n + p : n + p - 1, n2 = (a == 0 && !D.scalar) ? n + p - 1 : n + p;
            for (int i2 = 0; i2 < n2; ++i2)
                for (int i1 = 0; i1 < n1; ++i1) {
                    const int32_t g = D.dof[(((size_t)j * 2 + a) * nb + i2) * nb + i1];
                    if (g < 0 || own[g] >= 0) continue;
                    const int e1 = std::min(i1, n - 1), e2 = std::min(i2, n - 1);
                    own[g] = (j * SL + e2 / s) * SL + e1 / s;
                }
        }
    for (int64_t i = 0; i < N; ++i) IGE_REQUIRE(own[i] >= 0, "unknown without an owner leaf");
    // per leaf: its slot unknowns grouped by owner, (owner, sorted unknowns)
    std::vector<std::vector<std::pair<int32_t, std::vector<int32_t>>>> grp((size_t)nleaf);
    for (int t = 0; t < nleaf; ++t) {
        std::map<int32_t, std::vector<int32_t>> m;
        for (int k = 0; k < nF; ++k) {
            const int32_t g = B.leafdof[(size_t)t * nF + k];
            if (g >= 0) m[own[g]].push_back(g);
        }
        for (auto &kv : m) {
            std::sort(kv.second.begin(), kv.second.end());
            kv.second.erase(std::unique(kv.second.begin(), kv.second.end()), kv.second.end());
            grp[t].emplace_back(kv.first, std::move(kv.second));
        }
    }
    auto slice = [&](int leaf, int32_t owner) -> const std::vector<int32_t> & {
        for (const auto &g : grp[leaf])
            if (g.first == owner) return g.second;
        throw Status{IGE_EINVAL, "internal: owner slice not found"};
    };
    // off-diagonal owner blocks: for every row, the leaves that give it columns;
    // diagonal owner blocks: their unknowns
    std::map<std::pair<int32_t, int32_t>, std::map<int32_t, std::vector<int32_t>>> off;
    std::map<int32_t, std::vector<int32_t>> diag;
    for (int64_t b = 0; b < B.nblk(); ++b) {
        const int t = B.pair[2 * b], u = B.pair[2 * b + 1];
        for (const auto &gt : grp[t])
            for (const auto &gu : grp[u]) {
                const int32_t Tt = gt.first, Su = gu.first;
                if (Tt == Su) {
                    auto &dv = diag[Tt];
                    dv.insert(dv.end(), gt.second.begin(), gt.second.end());
                    dv.insert(dv.end(), gu.second.begin(), gu.second.end());
                } else if (Tt < Su) {
                    auto &rows = off[{Tt, Su}];
                    for (int32_t i : gt.second) rows[i].push_back(u);
                } else {
                    auto &rows = off[{Su, Tt}];
                    for (int32_t i : gu.second) rows[i].push_back(t);
                }
            }
    }
    auto add_sub = [&](const std::vector<int32_t> &rows, const std::vector<int32_t> &cols, bool sq) {
        C.nr.push_back((int32_t)rows.size());
        C.nc.push_back((int32_t)cols.size());
        C.sym.push_back(sq ? 1 : 0);
        const int32_t ld = (int32_t)((cols.size() + 3) / 4 * 4);
        C.nval = (C.nval + 15) / 16 * 16;
        C.val.push_back(C.nval);
        C.ld.push_back(ld);
        C.lst.push_back((int64_t)C.idx.size());
        C.idx.insert(C.idx.end(), rows.begin(), rows.end());
        C.idx.insert(C.idx.end(), cols.begin(), cols.end());
        C.nval += (int64_t)rows.size() * ld;
        C.distinct += sq ? (int64_t)rows.size() * ((int64_t)rows.size() + 1) / 2
                         : (int64_t)rows.size() * (int64_t)cols.size();
        C.maxn = std::max(C.maxn, (int)std::max(rows.size(), cols.size()));
    };
    // in owner order: the diagonal square of T, then its off-diagonal blocks (T, S > T)
    auto it = off.begin();
    for (int32_t Tt = 0; Tt < nleaf; ++Tt) {
        auto dt = diag.find(Tt);
        if (dt != diag.end()) {
            auto &v = dt->second;
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
            add_sub(v, v, true);
        }
        for (; it != off.end() && it->first.first == Tt; ++it) {
            const int32_t Su = it->first.second;
            // rows with the same set of column leaves form one rectangle
            std::map<std::vector<int32_t>, std::vector<int32_t>> byset;
            for (auto &rv : it->second) {
                auto &ls = rv.second;
                std::sort(ls.begin(), ls.end());
                ls.erase(std::unique(ls.begin(), ls.end()), ls.end());
                byset[ls].push_back(rv.first);
            }
            for (auto &kv : byset) {
                std::vector<int32_t> cols;
                for (int32_t leaf : kv.first) {
                    const auto &sl = slice(leaf, Su);
                    cols.insert(cols.end(), sl.begin(), sl.end());
                }
                std::sort(cols.begin(), cols.end());
                cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
                add_sub(kv.second, cols, false);
            }
        }
    }
    IGE_REQUIRE(C.idx.size() < ((size_t)1 << 31), "near field too large for 32-bit index lists");
    // work items and partial results
    const int RI = std::max(1, rows_per_item);
    for (int64_t k = 0; k < C.nsub(); ++k)
        for (int r0 = 0; r0 < C.nr[k]; r0 += RI) {
            const int r1 = std::min(C.nr[k], r0 + RI);
            C.wsub.push_back((int32_t)k);
            C.wr0.push_back(r0);
            C.wr1.push_back(r1);
            C.wpart.push_back(C.npart);
            C.npart += (r1 - r0) + C.nc[k];
        }
    IGE_REQUIRE(C.npart < ((int64_t)1 << 31), "near field too large for 32-bit partial indices");
    // launch order: the work items of at most 128 columns, then the wider ones (two
    // launches with different lane tiling), each largest first
    C.worder.resize(C.wsub.size());
    std::iota(C.worder.begin(), C.worder.end(), 0);
    std::stable_sort(C.worder.begin(), C.worder.end(), [&](int32_t a, int32_t b) {
        const bool na = C.nc[C.wsub[a]] <= 128, nb = C.nc[C.wsub[b]] <= 128;
        if (na != nb) return na;
        return (int64_t)(C.wr1[a] - C.wr0[a]) * C.nc[C.wsub[a]] > (int64_t)(C.wr1[b] - C.wr0[b]) * C.nc[C.wsub[b]];
    });
    C.nnarrow = 0;
    while (C.nnarrow < (int64_t)C.worder.size() && C.nc[C.wsub[C.worder[C.nnarrow]]] <= 128) ++C.nnarrow;
    // per unknown its partial results in ascending order
    std::vector<int64_t> cnt((size_t)N + 1, 0);
    auto visit = [&](auto &&emit) {
        for (size_t w = 0; w < C.wsub.size(); ++w) {
            const int k = C.wsub[w];
            const int32_t *rows = &C.idx[C.lst[k]], *cols = rows + C.nr[k];
            for (int r = C.wr0[w]; r < C.wr1[w]; ++r) emit(rows[r], C.wpart[w] + (r - C.wr0[w]));
            for (int c = 0; c < C.nc[k]; ++c) emit(cols[c], C.wpart[w] + (C.wr1[w] - C.wr0[w]) + c);
        }
    };
    visit([&](int32_t g, int64_t) { cnt[g + 1]++; });
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    C.red_ptr = cnt;
    C.red_idx.assign(cnt[N], 0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    visit([&](int32_t g, int64_t slot) { C.red_idx[fill[g]++] = (int32_t)slot; });
    // merge tables
    std::vector<int32_t> oc((size_t)N + 1, 0);
    for (size_t q = 0; q < B.leafdof.size(); ++q)
        if (B.leafdof[q] >= 0) oc[B.leafdof[q] + 1]++;
    for (int64_t i = 0; i < N; ++i) oc[i + 1] += oc[i];
    C.occ_ptr = oc;
    C.occ.assign(oc[N], 0);
    {
        std::vector<int32_t> f(oc.begin(), oc.end() - 1);
        for (size_t q = 0; q < B.leafdof.size(); ++q)
            if (B.leafdof[q] >= 0) C.occ[f[B.leafdof[q]]++] = (int32_t)q;   // ascending in q
    }
    std::vector<std::vector<std::pair<int32_t, int32_t>>> nbr((size_t)nleaf);
    for (int64_t b = 0; b < B.nblk(); ++b) {
        const int t = B.pair[2 * b], u = B.pair[2 * b + 1];
        nbr[t].push_back({u, (int32_t)(2 * b)});
        if (u != t) nbr[u].push_back({t, (int32_t)(2 * b + 1)});
    }
    C.np_ptr.assign((size_t)nleaf + 1, 0);
    for (int t = 0; t < nleaf; ++t) {
        std::sort(nbr[t].begin(), nbr[t].end());
        C.np_ptr[t + 1] = C.np_ptr[t] + (int32_t)nbr[t].size();
        for (const auto &e : nbr[t]) {
            C.np_leaf.push_back(e.first);
            C.np_code.push_back(e.second);
        }
    }
}

// ---------------------------------------------------------------------------
// singular element pairs (shared corner) with their reference frames
// ---------------------------------------------------------------------------
namespace {
const int kCorner[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};

// frame code: origin corner o (bit0 = o1, bit1 = o2), bit2 set when the first
// canonical axis runs along v
int frame_code(int origin, int towards_a2)
{
    const int o1 = kCorner[origin][0], o2 = kCorner[origin][1];
    const bool a2_along_v = kCorner[towards_a2][0] == o1;   // same u => differs in v
    const int swap = a2_along_v ? 0 : 1;                    // a1 along u iff a2 along v
    return o1 | (o2 << 1) | (swap << 2);
}
}  // namespace

void build_singular_pairs(std::vector<SingularPair> &S, std::vector<double> &corners, const Geometry &G,
                          const Discretisation &D, const Partition &T, const NearBlocks &B)
{
    const int n = D.n, s = T.s, SL = 1 << T.L;
    const std::vector<double> V = vertex_images(G, n);
    const size_t E = (size_t)D.P * n * n;
    corners.resize(E * 12);
    std::vector<double> cen(E * 3), rad(E);
    for (int j = 0; j < D.P; ++j)
        for (int e2 = 0; e2 < n; ++e2)
            for (int e1 = 0; e1 < n; ++e1) {
                const size_t e = ((size_t)j * n + e2) * n + e1;
                double c[3] = {0, 0, 0};
                for (int k = 0; k < 4; ++k) {
                    const double *v =
                        &V[(((size_t)j * (n + 1) + e2 + kCorner[k][1]) * (n + 1) + e1 + kCorner[k][0]) * 3];
                    for (int d = 0; d < 3; ++d) {
                        corners[e * 12 + k * 3 + d] = v[d];
                        c[d] += 0.25 * v[d];
                    }
                }
                double r = 0.0;
                for (int k = 0; k < 4; ++k) r = std::max(r, dist3(c, &corners[e * 12 + k * 3]));
                for (int d = 0; d < 3; ++d) cen[e * 3 + d] = c[d];
                rad[e] = r;
            }
    const double tol = 1e-9 * G.scale;
    S.clear();
    for (int64_t blk = 0; blk < B.nblk(); ++blk) {
        const int lt = B.pair[2 * blk], ls = B.pair[2 * blk + 1];
        const int jt = lt / (SL * SL), rt = lt % (SL * SL), jt2 = rt / SL, jt1 = rt % SL;
        const int js = ls / (SL * SL), rs = ls % (SL * SL), js2 = rs / SL, js1 = rs % SL;
        for (int a2 = 0; a2 < s; ++a2)
            for (int a1 = 0; a1 < s; ++a1) {
                const size_t e = ((size_t)jt * n + jt2 * s + a2) * n + jt1 * s + a1;
                for (int b2 = 0; b2 < s; ++b2)
                    for (int b1 = 0; b1 < s; ++b1) {
                        const size_t f = ((size_t)js * n + js2 * s + b2) * n + js1 * s + b1;
                        if (dist3(&cen[e * 3], &cen[f * 3]) > rad[e] + rad[f] + 2 * tol) continue;
                        int ti[4], si[4], ns = 0;
                        for (int x = 0; x < 4; ++x)
                            for (int y = 0; y < 4; ++y)
                                if (dist3(&corners[e * 12 + x * 3], &corners[f * 12 + y * 3]) <= tol) {
                                    ti[ns] = x;
                                    si[ns] = y;
                                    ++ns;
                                }
                        if (ns == 0) continue;
                        SingularPair sp{(int32_t)e, (int32_t)f, 0, 0, 0, (int32_t)blk};
                        if (ns == 4) {
                            IGE_REQUIRE(e == f, "distinct elements share all corners");
                            sp.kind = 1;
                        } else if (ns == 2) {
                            IGE_REQUIRE(((ti[0] - ti[1]) & 3) != 2 && ((si[0] - si[1]) & 3) != 2,
                                        "elements share two opposite corners");
                            sp.kind = 2;
                            sp.fa = frame_code(ti[0], ti[1]);
                            sp.fb = frame_code(si[0], si[1]);
                        } else if (ns == 1) {
                            sp.kind = 3;
                            sp.fa = frame_code(ti[0], (ti[0] + 3) & 3);
                            sp.fb = frame_code(si[0], (si[0] + 3) & 3);
                        } else {
                            IGE_REQUIRE(false, "elements share three corners");
                        }
                        S.push_back(sp);
                    }
            }
    }
}

// ---------------------------------------------------------------------------
// far-field tables: 1-D cluster moments of the splines and transfer matrices
// ---------------------------------------------------------------------------
void build_far_tables(FarTables &F, const Discretisation &D, const Partition &T, const std::vector<int> &ql)
{
    IGE_REQUIRE((int)ql.size() == T.L + 1, "one interpolation degree per level");
    int q = 0;
    for (int v : ql) {
        IGE_REQUIRE(v >= 1 && v + 1 <= kMaxQ1, "interpolation degrees must be 1..15");
        q = std::max(q, v);
    }
    const int p = D.p, n = D.n, s = T.s, S = 1 << T.L;
    const double h = 1.0 / n, H = 1.0 / S;
    F.q = q;
    F.Q1 = q + 1;
    F.rowlen = s + p;
    F.ql = ql;
    F.varq = false;
    for (int v : ql) F.varq = F.varq || v != q;
    F.xn.resize(q + 1);
    chebyshev01(q, F.xn.data());
    // per level: its nodes, and the restriction from the degree-q nodes
    F.xnl.assign((size_t)(T.L + 1) * kMaxQ1, 0.0);
    F.R.assign((size_t)(T.L + 1) * F.Q1 * F.Q1, 0.0);
    for (int l = 0; l <= T.L; ++l) {
        chebyshev01(ql[l], &F.xnl[(size_t)l * kMaxQ1]);
        for (int nn = 0; nn <= q; ++nn) {
            double Lm[kMaxQ1];
            lagrange_bary(ql[l], &F.xnl[(size_t)l * kMaxQ1], F.xn[nn], Lm);
            for (int mm = 0; mm <= ql[l]; ++mm) F.R[((size_t)l * F.Q1 + nn) * F.Q1 + mm] = Lm[mm];
        }
    }
    const int ng = (q + p) / 2 + 1;    // exact for the degree q + p moment integrands
    std::vector<double> gx(ng), gw(ng);
    gauss_legendre01(ng, gx.data(), gw.data());
    F.Mp.assign((size_t)S * F.Q1 * F.rowlen, 0.0);
    F.Mq.assign((size_t)S * F.Q1 * F.rowlen, 0.0);
    F.Mdp.assign((size_t)S * F.Q1 * F.rowlen, 0.0);
    auto bern = [](int deg, double x, double *B, double *Dd) {
        for (int a = 0; a <= deg; ++a) {
            B[a] = binom(deg, a) * std::pow(x, a) * std::pow(1.0 - x, deg - a);
            double d = 0.0;
            if (deg > 0) {
                const double lo = (a >= 1) ? binom(deg - 1, a - 1) * std::pow(x, a - 1) * std::pow(1.0 - x, deg - a) : 0.0;
                const double hi = (a <= deg - 1) ? binom(deg - 1, a) * std::pow(x, a) * std::pow(1.0 - x, deg - 1 - a) : 0.0;
                d = deg * (lo - hi);
            }
            Dd[a] = d;
        }
    };
    for (int k = 0; k < S; ++k)
        for (int el = 0; el < s; ++el) {
            const int e = k * s + el;
            for (int g = 0; g < ng; ++g) {
                const double u = (e + gx[g]) * h, w = gw[g] * h;
                double Lm[kMaxQ1];
                lagrange_bary(q, F.xn.data(), (u - k * H) / H, Lm);
                double Bp[kMaxP + 2], dBp[kMaxP + 2], Bq[kMaxP + 2], dBq[kMaxP + 2];
                bern(p, gx[g], Bp, dBp);
                bern(p - 1, gx[g], Bq, dBq);
                for (int t = 0; t <= p; ++t) {   // b^p_{e+t}
                    double v = 0.0, dv = 0.0;
                    for (int a = 0; a <= p; ++a) {
                        v += D.ext_p[((size_t)e * (p + 1) + t) * (p + 1) + a] * Bp[a];
                        dv += D.ext_p[((size_t)e * (p + 1) + t) * (p + 1) + a] * dBp[a];
                    }
                    dv /= h;
                    const int il = el + t;
                    for (int mm = 0; mm <= q; ++mm) {
                        F.Mp[((size_t)k * F.Q1 + mm) * F.rowlen + il] += w * Lm[mm] * v;
                        F.Mdp[((size_t)k * F.Q1 + mm) * F.rowlen + il] += w * Lm[mm] * dv;
                    }
                }
                for (int t = 0; t < p; ++t) {   // b^{p-1}_{e+t}
                    double v = 0.0;
                    for (int a = 0; a < p; ++a) v += D.ext_q[((size_t)e * p + t) * p + a] * Bq[a];
                    const int il = el + t;
                    for (int mm = 0; mm <= q; ++mm) F.Mq[((size_t)k * F.Q1 + mm) * F.rowlen + il] += w * Lm[mm] * v;
                }
            }
        }
    F.T0.assign((size_t)F.Q1 * F.Q1, 0.0);
    F.T1.assign((size_t)F.Q1 * F.Q1, 0.0);
    for (int nn = 0; nn <= q; ++nn) {
        double L0[kMaxQ1], L1[kMaxQ1];
        lagrange_bary(q, F.xn.data(), 0.5 * F.xn[nn], L0);
        lagrange_bary(q, F.xn.data(), 0.5 * (F.xn[nn] + 1.0), L1);
        for (int mm = 0; mm <= q; ++mm) {
            F.T0[nn * F.Q1 + mm] = L0[mm];
            F.T1[nn * F.Q1 + mm] = L1[mm];
        }
    }
}

}  // namespace ige
