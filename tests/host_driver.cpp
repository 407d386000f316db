// Host-side driver of the igaefie C ABI for the sanitizer tests (no device calls):
// host-only contexts, geometry validation, operator planning (unknowns, cluster and
// block-cluster trees, near-field layouts) and the error paths, first on one thread,
// then on several threads at once (one context per thread, and one geometry shared by
// all threads, which planning only reads).
//
// usage: host_driver <geometry file> <threads>
// geometry file: int32 P, int32 degree[2P], int32 n_ctrl[2P], int64 n_knots,
// double knots[n_knots], int64 n_ctrl_total, double ctrl[n_ctrl_total][4]
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../include/igaefie.h"

namespace {

struct GeomData {
    int P = 0;
    std::vector<int> deg, nctrl;
    std::vector<double> knots, ctrl;
};

bool read_geom(const char *path, GeomData &g)
{
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    int32_t P = 0;
    int64_t nk = 0, nc = 0;
    bool ok = std::fread(&P, 4, 1, f) == 1 && P > 0 && P < 10000;
    if (ok) {
        g.P = P;
        g.deg.resize(2 * P);
        g.nctrl.resize(2 * P);
        ok = std::fread(g.deg.data(), 4, 2 * P, f) == (size_t)(2 * P) &&
             std::fread(g.nctrl.data(), 4, 2 * P, f) == (size_t)(2 * P) && std::fread(&nk, 8, 1, f) == 1;
    }
    if (ok) {
        g.knots.resize(nk);
        ok = std::fread(g.knots.data(), 8, nk, f) == (size_t)nk && std::fread(&nc, 8, 1, f) == 1;
    }
    if (ok) {
        g.ctrl.resize(4 * nc);
        ok = std::fread(g.ctrl.data(), 8, 4 * nc, f) == (size_t)(4 * nc);
    }
    std::fclose(f);
    return ok;
}

int g_fail = 0;
#define CHECK(c)                                                                          \
    do {                                                                                  \
        if (!(c)) {                                                                       \
            std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #c,      \
                         ige_last_error());                                               \
            __atomic_add_fetch(&g_fail, 1, __ATOMIC_RELAXED);                             \
        }                                                                                 \
    } while (0)

// plan one operator and read everything a planned operator answers
void plan_one(ige_geom geom, int p, int level, double kappa, int q, double eta, int d, double cap, int P,
              int kind = IGE_OP_EFIE)
{
    ige_params prm{p, level, kappa, q, eta, 5, 5, d, 0, cap, kind};
    ige_op op = nullptr;
    CHECK(ige_op_plan(geom, &prm, &op) == IGE_OK);
    if (!op) return;
    ige_op_info_t info{};
    CHECK(ige_op_info(op, &info) == IGE_OK);
    const int64_t n = (int64_t)1 << level, nb = n + p;
    CHECK(info.n_dof == (kind == IGE_OP_SCALAR ? (int64_t)P * nb * nb : 2 * (int64_t)P * (n + p - 1) * (n + p - 1)));
    CHECK(info.near_distinct > 0 && info.near_distinct <= info.n_dof * (info.n_dof + 1) / 2);
    std::vector<int32_t> dof((size_t)P * 2 * nb * nb), far((size_t)3 * info.far_pairs + 1),
        near((size_t)2 * info.near_leaf_pairs + 1);
    std::vector<int8_t> sgn(dof.size());
    CHECK(ige_op_dofmap(op, dof.data(), sgn.data()) == IGE_OK);
    CHECK(ige_op_partition(op, far.data(), near.data()) == IGE_OK);
    int64_t used = 0;
    for (int32_t v : dof) used += v >= 0 && v < info.n_dof;
    CHECK(used >= info.n_dof);
    // a planned operator refuses device work
    std::vector<ige_c64> x((size_t)info.n_dof), y(x.size());
    CHECK(ige_apply(op, 1, x.data(), y.data(), IGE_HOST) == IGE_EINVAL);
    CHECK(std::strlen(ige_last_error()) > 0);
    CHECK(ige_op_destroy(op) == IGE_OK);
}

void error_paths(ige_geom geom)
{
    ige_op op = nullptr;
    ige_params bad{0, 2, 1.0, 8, 1.0, 5, 5, -1, 0, 0.0};
    CHECK(ige_op_plan(geom, &bad, &op) == IGE_EINVAL && op == nullptr);
    CHECK(std::string(ige_last_error()).find("p must") != std::string::npos);
    ige_params bad2{2, 2, -1.0, 8, 1.0, 5, 5, -1, 0, 0.0};
    CHECK(ige_op_plan(geom, &bad2, &op) == IGE_EINVAL);
    CHECK(std::string(ige_last_error()).find("kappa") != std::string::npos);
    ige_params bad3{2, 2, 1.0, 8, 1.0, 5, 5, -1, 0, -2.0};
    CHECK(ige_op_plan(geom, &bad3, &op) == IGE_EINVAL);
    ige_params bad4{2, 2, 1.0, 8, 1.0, 5, 5, -1, 0, 0.0, 7};
    CHECK(ige_op_plan(geom, &bad4, &op) == IGE_EINVAL);
    CHECK(std::string(ige_last_error()).find("kind") != std::string::npos);
    CHECK(ige_op_plan(nullptr, &bad, &op) == IGE_EINVAL);
    ige_params ok{1, 1, 1.0, 4, 1.0, 5, 5, -1, 0, 0.0};
    CHECK(ige_op_plan(geom, &ok, &op) == IGE_OK);   // success clears the error text
    CHECK(std::strlen(ige_last_error()) == 0);
    if (op) ige_op_destroy(op);
}

void worker(const GeomData *gd, ige_geom shared, int id)
{
    ige_ctx ctx = nullptr;
    CHECK(ige_ctx_create(-1, nullptr, &ctx) == IGE_OK);
    ige_geom own = nullptr;
    CHECK(ige_geom_create(ctx, gd->P, gd->deg.data(), gd->nctrl.data(), gd->knots.data(), gd->ctrl.data(), &own) ==
          IGE_OK);
    for (int k = 0; k < 3; ++k) {
        const int p = 1 + (id + k) % 4;
        plan_one(own, p, 2 + (id + k) % 2, 2.0 + id, 6, 1.0, 1, 0.0, gd->P);
        plan_one(shared, 1 + (id + k + 1) % 3, 3, 8.0, 8, 1.6, 1 + k % 2, (k == 2) ? 8.0 : 0.0, gd->P);
        plan_one(own, 1 + (id + k) % 4, 3, 4.0, 6, 1.0, 1, 0.0, gd->P, IGE_OP_SCALAR);
        error_paths(own);
    }
    CHECK(ige_geom_destroy(own) == IGE_OK);
    CHECK(ige_ctx_destroy(ctx) == IGE_OK);
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc < 3) {
        std::fprintf(stderr, "usage: %s <geometry file> <threads>\n", argv[0]);
        return 2;
    }
    GeomData gd;
    if (!read_geom(argv[1], gd)) {
        std::fprintf(stderr, "cannot read %s\n", argv[1]);
        return 2;
    }
    const int nt = std::atoi(argv[2]);
    ige_ctx ctx = nullptr;
    CHECK(ige_ctx_create(-1, nullptr, &ctx) == IGE_OK);
    ige_geom geom = nullptr;
    CHECK(ige_geom_create(ctx, gd.P, gd.deg.data(), gd.nctrl.data(), gd.knots.data(), gd.ctrl.data(), &geom) == IGE_OK);
    // malformed geometry: a negative weight and a missing patch
    std::vector<double> badc = gd.ctrl;
    badc[7] = -1.0;
    ige_geom g2 = nullptr;
    CHECK(ige_geom_create(ctx, gd.P, gd.deg.data(), gd.nctrl.data(), gd.knots.data(), badc.data(), &g2) == IGE_EINVAL);
    CHECK(ige_geom_create(ctx, gd.P - 1, gd.deg.data(), gd.nctrl.data(), gd.knots.data(), gd.ctrl.data(), &g2) ==
          IGE_EINVAL);
    // one thread: every degree, several levels, leaf depths, the dense case and the cap
    for (int p = 1; p <= 4; ++p)
        for (int m = 0; m <= 4; ++m) plan_one(geom, p, m, 4.0, 6, m % 2 ? 1.6 : 1.0, -1, 0.0, gd.P);
    plan_one(geom, 2, 4, 16.0, 8, 1.6, 2, 8.0, gd.P);
    plan_one(geom, 2, 3, 1.0, 8, 0.0, -1, 0.0, gd.P);
    error_paths(geom);
    // several threads at once
    std::vector<std::thread> th;
    for (int i = 0; i < nt; ++i) th.emplace_back(worker, &gd, geom, i);
    for (auto &t : th) t.join();
    // a context outlives what was made on it
    CHECK(ige_ctx_destroy(ctx) == IGE_EINVAL);
    CHECK(ige_geom_destroy(geom) == IGE_OK);
    CHECK(ige_ctx_destroy(ctx) == IGE_OK);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host driver: all checks passed (%d threads)\n", nt);
    return 0;
}
