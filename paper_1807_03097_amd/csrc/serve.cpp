// Serving: many independent scattering solves (geometry, discretisation,
// wavenumber and one or several incident plane waves each) on one device.
//
// A server owns n_workers host threads; each has its own context, i.e. its own HIP
// stream, so the kernels of several requests share the device.  Requests wait in
// arrival order and are admitted first-fit by their planned device footprint
// against a memory budget; a request may overtake the oldest waiting one only while
// that one has waited less than kMaxBypass seconds, which bounds its delay.  A
// worker assembles the operator on its stream, forms the right-hand sides, runs GMRES
// on all of them at once (the batched kernels from two waves on) and copies the
// solutions to host memory, then frees the operator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "op.hpp"

namespace {

constexpr double kMaxBypass = 1.0;   // seconds

struct SrvReq {
    int64_t ticket = 0;
    const ige_geom_s *geom = nullptr;
    ige_params prm{};
    int nw = 1;                  // plane waves (right-hand sides)
    std::vector<double> dir;     // [nw][3]
    std::vector<ige_c64> pol;    // [nw][3]
    ige_solve_opts opts{};
    size_t footprint = 0;
    int64_t n_dof = 0;
    int state = 0;   // 0 queued, 1 running, 2 finished
    int rc = 0;
    std::string err;
    int iters = 0;
    double relres = 0.0;
    double t_submit = 0.0, t_start = 0.0, t_done = 0.0, assemble_s = 0.0, solve_s = 0.0;
    std::vector<ige_c64> x;
};

}  // namespace

struct ige_srv_s {
    ige_ctx parent = nullptr;
    int device = 0;
    size_t budget = 0, in_use = 0;
    std::chrono::steady_clock::time_point origin;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SrvReq *> queue;
    std::map<int64_t, std::unique_ptr<SrvReq>> all;
    std::vector<std::thread> workers;
    int64_t next_ticket = 1;
    bool stop = false;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - origin).count();
    }

    // first request (arrival order) that fits next to the running ones; the oldest
    // one is overtaken only while it has waited less than kMaxBypass
    SrvReq *pick()
    {
        if (queue.empty()) return nullptr;
        const double t = now();
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            if (in_use + (*it)->footprint <= budget) {
                SrvReq *r = *it;
                queue.erase(it);
                return r;
            }
            if (it == queue.begin() && t - (*it)->t_submit >= kMaxBypass) return nullptr;
        }
        return nullptr;
    }

    void run(SrvReq *r, ige_ctx wctx)
    {
        const double t0 = now();
        ige_op op = nullptr;
        try {
            op = ige::assemble_on(wctx, r->geom, r->prm);
            const double t1 = now();
            r->assemble_s = t1 - t0;
            const int64_t N = op->D.N;
            std::vector<ige_c64> f((size_t)N * r->nw);
            r->x.assign((size_t)N * r->nw, ige_c64{0.0, 0.0});
            int rc = ige_rhs_plane_wave(op, r->nw, r->dir.data(), r->pol.data(), f.data(), IGE_HOST);
            if (rc != IGE_OK) throw ige::Status{rc, ige_last_error()};
            std::vector<ige_solve_stats> st((size_t)r->nw);
            rc = ige_solve(op, r->nw, f.data(), r->x.data(), IGE_HOST, &r->opts, st.data());
            if (rc != IGE_OK && rc != IGE_ENOTCONV) throw ige::Status{rc, ige_last_error()};
            r->rc = rc;
            for (const auto &c : st) {   // the slowest wave
                r->iters = std::max(r->iters, c.iters);
                r->relres = std::max(r->relres, c.relres);
            }
            r->solve_s = now() - t1;
        } catch (const ige::Status &e) {
            r->rc = e.code;
            r->err = e.msg;
        } catch (const std::bad_alloc &) {
            r->rc = IGE_ENOMEM;
            r->err = "host allocation failed";
        } catch (const std::exception &e) {
            r->rc = IGE_EINVAL;
            r->err = std::string("request failed: ") + e.what();
        } catch (...) {
            // nothing may escape a worker thread (that would end the process)
            r->rc = IGE_EINVAL;
            r->err = "request failed with an unknown exception";
        }
        if (op) ige_op_destroy(op);
    }

    void worker_main()
    {
        ige_ctx wctx = nullptr;
        const int rc = ige_ctx_create(device, nullptr, &wctx);
        for (;;) {
            SrvReq *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return (r = pick()) != nullptr || (stop && queue.empty()); });
                if (!r) break;
                in_use += r->footprint;
                r->state = 1;
                r->t_start = now();
            }
            if (rc == IGE_OK) {
                run(r, wctx);   // reports every failure in r (catches all exceptions)
            } else {
                r->rc = rc;
                r->err = "worker context creation failed";
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= r->footprint;
                r->t_done = now();
                r->state = 2;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
        if (wctx) ige_ctx_destroy(wctx);
    }
};

namespace {

void fill_stats(const SrvReq &r, ige_srv_stats *st)
{
    if (!st) return;
    st->state = r.state;
    st->rc = r.rc;
    st->iters = r.iters;
    st->relres = r.relres;
    st->n_dof = r.n_dof;
    st->footprint = r.footprint;
    st->t_submit = r.t_submit;
    st->t_start = r.t_start;
    st->t_done = r.t_done;
    st->assemble_s = r.assemble_s;
    st->solve_s = r.solve_s;
    st->n_waves = r.nw;
}

template <typename F>
int srv_guard(F &&f)
{
    try {
        f();
        return IGE_OK;
    } catch (const ige::Status &e) {
        ige::set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        ige::set_error("host allocation failed");
        return IGE_ENOMEM;
    } catch (const std::exception &e) {
        ige::set_error(e.what());
        return IGE_EINVAL;
    } catch (...) {
        ige::set_error("unknown exception");
        return IGE_EINVAL;
    }
}

}  // namespace

extern "C" {

int ige_srv_create(ige_ctx ctx, int n_workers, size_t hbm_budget, ige_srv *out)
{
    return srv_guard([&] {
        IGE_REQUIRE(ctx && out, "null argument");
        IGE_REQUIRE(ctx->device >= 0, "serving needs a device context");
        IGE_REQUIRE(n_workers >= 1 && n_workers <= 64, "n_workers must be 1..64");
        auto srv = std::make_unique<ige_srv_s>();
        srv->parent = ctx;
        srv->device = ctx->device;
        IGE_HIP(hipSetDevice(ctx->device));
        if (hbm_budget == 0) {
            size_t fr = 0, tot = 0;
            IGE_HIP(hipMemGetInfo(&fr, &tot));
            hbm_budget = fr / 10 * 8;
        }
        srv->budget = hbm_budget;
        srv->origin = std::chrono::steady_clock::now();
        ige_srv_s *s = srv.get();
        for (int i = 0; i < n_workers; ++i) s->workers.emplace_back([s] { s->worker_main(); });
        *out = srv.release();
    });
}

int ige_srv_submit(ige_srv srv, ige_geom geom, const ige_params *prm, const double *dir, const ige_c64 *pol,
                   const ige_solve_opts *opts, int64_t *ticket)
{
    return ige_srv_submit_waves(srv, geom, prm, 1, dir, pol, opts, ticket);
}

int ige_srv_submit_waves(ige_srv srv, ige_geom geom, const ige_params *prm, int n_waves, const double *dir,
                         const ige_c64 *pol, const ige_solve_opts *opts, int64_t *ticket)
{
    return srv_guard([&] {
        IGE_REQUIRE(srv && geom && prm && dir && pol && opts && ticket, "null argument");
        IGE_REQUIRE(opts->restart >= 1 && opts->maxit >= 0, "bad solve options");
        IGE_REQUIRE(n_waves >= 1 && n_waves <= 4096, "n_waves must be 1..4096");
        auto r = std::make_unique<SrvReq>();
        r->geom = geom;
        r->prm = *prm;
        r->nw = n_waves;
        r->dir.assign(dir, dir + 3 * (size_t)n_waves);
        r->pol.assign(pol, pol + 3 * (size_t)n_waves);
        r->opts = *opts;
        // footprint from the host plan of the operator
        ige_op planned = nullptr;
        int rc = ige_op_plan(geom, prm, &planned);
        if (rc != IGE_OK) throw ige::Status{rc, ige_last_error()};
        r->footprint = ige::planned_device_bytes(planned, opts->restart, n_waves, opts);
        r->n_dof = planned->D.N;
        ige_op_destroy(planned);
        std::lock_guard<std::mutex> lk(srv->mu);
        IGE_REQUIRE(!srv->stop, "server is shutting down");
        if (r->footprint > srv->budget)
            throw ige::Status{IGE_ENOMEM, "request footprint exceeds the server's memory budget"};
        r->ticket = srv->next_ticket++;
        r->t_submit = srv->now();
        *ticket = r->ticket;
        srv->queue.push_back(r.get());
        srv->all[r->ticket] = std::move(r);
        srv->cv_work.notify_one();
    });
}

int ige_srv_poll(ige_srv srv, int64_t ticket, ige_srv_stats *stats)
{
    return srv_guard([&] {
        IGE_REQUIRE(srv, "null server");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->all.find(ticket);
        IGE_REQUIRE(it != srv->all.end(), "unknown ticket");
        fill_stats(*it->second, stats);
    });
}

int ige_srv_wait(ige_srv srv, int64_t ticket, ige_srv_stats *stats)
{
    return srv_guard([&] {
        IGE_REQUIRE(srv, "null server");
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->all.find(ticket);
        IGE_REQUIRE(it != srv->all.end(), "unknown ticket");
        SrvReq *r = it->second.get();
        srv->cv_done.wait(lk, [&] { return r->state == 2; });
        fill_stats(*r, stats);
    });
}

int ige_srv_result(ige_srv srv, int64_t ticket, ige_c64 *x, int64_t n)
{
    return srv_guard([&] {
        IGE_REQUIRE(srv && x, "null argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->all.find(ticket);
        IGE_REQUIRE(it != srv->all.end(), "unknown ticket");
        const SrvReq &r = *it->second;
        IGE_REQUIRE(r.state == 2, "request not finished");
        IGE_REQUIRE(r.rc == IGE_OK || r.rc == IGE_ENOTCONV, r.err.empty() ? "request failed" : r.err.c_str());
        IGE_REQUIRE(n == (int64_t)r.x.size(), "x has the wrong length");
        std::copy(r.x.begin(), r.x.end(), x);
    });
}

int ige_srv_destroy(ige_srv srv)
{
    return srv_guard([&] {
        if (!srv) return;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->cv_work.notify_all();
        for (auto &t : srv->workers) t.join();
        delete srv;
    });
}

}  // extern "C"
