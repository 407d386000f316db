// Serving: many scattering solves (geometry, discretisation, wavenumber and one or
// several incident plane waves each) on one device, as they arrive.
//
// A server owns n_workers host threads; each has its own context, i.e. its own HIP
// stream, so the kernels of several requests share the device.  Requests wait in
// arrival order and are admitted first-fit by their planned device footprint
// against a memory budget; a request may overtake the oldest waiting one only while
// that one has waited less than kMaxBypass seconds, which bounds its delay.
//
// Continuous batching: when a worker takes a request, the other waiting requests on
// the same operator (same geometry handle, parameters and solve options) join it, up
// to max_merge plane waves in all, and all their waves are solved together as one
// many-column system (every kernel value and block entry is read once per column
// chunk); the solutions are split back per request.  A worker keeps the operator of
// its last request resident on the device (cluster trees, near-field blocks, moment
// tables and its Krylov workspace) and prefers waiting requests on that operator, so
// a stream of requests on one object is assembled once.  Resident operators count
// against the budget and are freed when a waiting request needs their memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
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
constexpr int kMergeDefault = 64;    // plane waves of one merged solve

struct SrvReq {
    int64_t ticket = 0;
    const ige_geom_s *geom = nullptr;
    ige_params prm{};
    int nw = 1;                  // plane waves (right-hand sides)
    std::vector<double> dir;     // [nw][3]
    std::vector<ige_c64> pol;    // [nw][3]
    ige_solve_opts opts{};
    size_t footprint = 0;        // planned device bytes of this request alone
    size_t fp_merged = 0;        // planned device bytes of a merged solve of max_merge waves
    size_t fp_operator = 0;      // of which the assembled operator (resident between requests)
    int64_t n_dof = 0;
    int state = 0;   // 0 queued, 1 running, 2 finished
    int rc = 0;
    std::string err;
    int iters = 0;
    double relres = 0.0;
    double t_submit = 0.0, t_start = 0.0, t_done = 0.0, assemble_s = 0.0, solve_s = 0.0;
    int merged = 1;              // requests solved together with this one (itself included)
    bool reused = false;         // ran on a resident operator (no assembly)
    std::vector<ige_c64> x;
};

bool same_operator(const SrvReq &a, const SrvReq &b)
{
    return a.geom == b.geom && std::memcmp(&a.prm, &b.prm, sizeof(ige_params)) == 0;
}
bool same_solve(const SrvReq &a, const SrvReq &b)
{
    return same_operator(a, b) && std::memcmp(&a.opts, &b.opts, sizeof(ige_solve_opts)) == 0;
}

// the operator a worker keeps resident after its last request
struct Resident {
    ige_op op = nullptr;
    const ige_geom_s *geom = nullptr;
    ige_params prm{};
    size_t bytes = 0;            // counted in the server's in_use
};

}  // namespace

struct ige_srv_s {
    ige_ctx parent = nullptr;
    int device = 0;
    size_t budget = 0, in_use = 0;
    int max_merge = kMergeDefault;
    std::chrono::steady_clock::time_point origin;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SrvReq *> queue;
    std::map<int64_t, std::unique_ptr<SrvReq>> all;
    std::vector<std::thread> workers;
    std::vector<Resident> resident;   // per worker
    int64_t next_ticket = 1;
    bool stop = false;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - origin).count();
    }

    // bytes a group led by r needs beyond what worker w already holds for it
    size_t need(const SrvReq *r, int w, bool merged) const
    {
        const size_t fp = merged ? r->fp_merged : r->footprint;
        const Resident &R = resident[w];
        const bool hit = R.op && R.geom == r->geom && std::memcmp(&R.prm, &r->prm, sizeof(ige_params)) == 0;
        return hit ? fp - std::min(fp, std::min(R.bytes, r->fp_operator)) : fp;
    }

    // Worker w picks its next group (called with mu held): a waiting request on its
    // resident operator first, else the first request (arrival order) that fits next to
    // the running ones, the oldest one overtaken only while it has waited less than
    // kMaxBypass.  Requests with the same operator and solve options join the group.
    // A resident operator that is not needed is dropped (to *drop, freed by the caller
    // outside the lock) when the oldest waiting request does not fit.
    std::vector<SrvReq *> pick(int w, ige_op *drop)
    {
        std::vector<SrvReq *> grp;
        if (queue.empty()) return grp;
        const double t = now();
        Resident &R = resident[w];
        auto fits = [&](const SrvReq *r, bool merged) {
            const size_t own = (R.op && !(R.geom == r->geom && std::memcmp(&R.prm, &r->prm, sizeof(ige_params)) == 0))
                                   ? R.bytes : 0;   // an unrelated resident operator is dropped on start
            return in_use - own + need(r, w, merged) <= budget;
        };
        auto it = queue.end();
        if (R.op && t - queue.front()->t_submit < kMaxBypass)
            for (auto jt = queue.begin(); jt != queue.end(); ++jt)
                if ((*jt)->geom == R.geom && std::memcmp(&(*jt)->prm, &R.prm, sizeof(ige_params)) == 0 &&
                    fits(*jt, false)) {
                    it = jt;
                    break;
                }
        if (it == queue.end())
            for (auto jt = queue.begin(); jt != queue.end(); ++jt) {
                if (fits(*jt, false)) {
                    it = jt;
                    break;
                }
                if (jt == queue.begin() && t - (*jt)->t_submit >= kMaxBypass) break;
            }
        if (it == queue.end()) {
            // the oldest request waits for memory: give back this worker's resident operator
            if (R.op) {
                in_use -= R.bytes;
                *drop = R.op;
                R = Resident{};
                cv_work.notify_all();   // the others may free theirs too
            }
            return grp;
        }
        SrvReq *lead = *it;
        queue.erase(it);
        grp.push_back(lead);
        // requests on the same operator with the same options join, while a solve of
        // max_merge waves still fits
        int waves = lead->nw;
        if (max_merge > 1 && fits(lead, true))
            for (auto jt = queue.begin(); jt != queue.end();) {
                if (same_solve(**jt, *lead) && waves + (*jt)->nw <= max_merge) {
                    waves += (*jt)->nw;
                    grp.push_back(*jt);
                    jt = queue.erase(jt);
                } else {
                    ++jt;
                }
            }
        return grp;
    }

    // Solve a group on the worker's context: assemble (or reuse the resident operator),
    // right-hand sides of all waves, one GMRES on all columns, results split per request.
    // Every failure is reported in the requests (all exceptions caught).
    void run(std::vector<SrvReq *> &grp, ige_ctx wctx, int w, ige_op &keep)
    {
        SrvReq *lead = grp[0];
        const double t0 = now();
        ige_op op = nullptr;
        std::string err;
        int rc = IGE_OK;
        try {
            Resident &R = resident[w];
            if (R.op && R.geom == lead->geom && std::memcmp(&R.prm, &lead->prm, sizeof(ige_params)) == 0) {
                op = R.op;   // already counted: its bytes move into the group's footprint
                for (auto *r : grp) r->reused = true;
            } else {
                op = ige::assemble_on(wctx, lead->geom, lead->prm);
            }
            const double t1 = now();
            int nw = 0;
            for (auto *r : grp) nw += r->nw;
            const int64_t N = op->D.N;
            std::vector<double> dir;
            std::vector<ige_c64> pol;
            for (auto *r : grp) {
                dir.insert(dir.end(), r->dir.begin(), r->dir.end());
                pol.insert(pol.end(), r->pol.begin(), r->pol.end());
            }
            std::vector<ige_c64> f((size_t)N * nw), x((size_t)N * nw, ige_c64{0.0, 0.0});
            int rr = ige_rhs_plane_wave(op, nw, dir.data(), pol.data(), f.data(), IGE_HOST);
            if (rr != IGE_OK) throw ige::Status{rr, ige_last_error()};
            std::vector<ige_solve_stats> st((size_t)nw);
            rr = ige_solve(op, nw, f.data(), x.data(), IGE_HOST, &lead->opts, st.data());
            if (rr != IGE_OK && rr != IGE_ENOTCONV) throw ige::Status{rr, ige_last_error()};
            const double t2 = now();
            int c0 = 0;
            for (auto *r : grp) {
                r->x.assign(x.begin() + (size_t)c0 * N, x.begin() + (size_t)(c0 + r->nw) * N);
                bool conv = true;
                for (int c = c0; c < c0 + r->nw; ++c) {   // the slowest wave of the request
                    r->iters = std::max(r->iters, st[c].iters);
                    r->relres = std::max(r->relres, st[c].relres);
                    conv = conv && st[c].relres <= lead->opts.tol;
                }
                r->rc = (rr == IGE_ENOTCONV && !conv) ? IGE_ENOTCONV : IGE_OK;
                r->assemble_s = r->reused ? 0.0 : t1 - t0;
                r->solve_s = t2 - t1;
                r->merged = (int)grp.size();
                c0 += r->nw;
            }
            keep = op;
            return;
        } catch (const ige::Status &e) {
            rc = e.code;
            err = e.msg;
        } catch (const std::bad_alloc &) {
            rc = IGE_ENOMEM;
            err = "host allocation failed";
        } catch (const std::exception &e) {
            rc = IGE_EINVAL;
            err = std::string("request failed: ") + e.what();
        } catch (...) {
            // nothing may escape a worker thread (that would end the process)
            rc = IGE_EINVAL;
            err = "request failed with an unknown exception";
        }
        for (auto *r : grp) {
            r->rc = rc;
            r->err = err;
        }
        keep = op;   // kept only if it is healthy (see worker_main)
    }

    void worker_main(int w)
    {
        ige_ctx wctx = nullptr;
        const int crc = ige_ctx_create(device, nullptr, &wctx);
        for (;;) {
            std::vector<SrvReq *> grp;
            ige_op drop = nullptr, old = nullptr;
            size_t held = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    grp = pick(w, &drop);
                    // a dropped resident operator is freed at once, outside the lock (its
                    // bytes already left in_use, so the memory must follow)
                    return drop || !grp.empty() || (stop && queue.empty());
                });
                if (!grp.empty()) {
                    Resident &R = resident[w];
                    const bool hit = R.op && R.geom == grp[0]->geom &&
                                     std::memcmp(&R.prm, &grp[0]->prm, sizeof(ige_params)) == 0;
                    if (R.op && !hit) {   // an unrelated resident operator makes room
                        in_use -= R.bytes;
                        old = R.op;
                        R = Resident{};
                    }
                    held = grp.size() > 1 ? grp[0]->fp_merged : grp[0]->footprint;
                    if (hit) {   // its resident bytes become part of the group's footprint
                        in_use -= R.bytes;
                        R.bytes = 0;
                    }
                    in_use += held;
                    const double t = now();
                    for (auto *r : grp) {
                        r->state = 1;
                        r->t_start = t;
                    }
                }
            }
            if (drop) ige_op_destroy(drop);
            if (old) ige_op_destroy(old);
            if (grp.empty()) {
                if (drop) continue;
                break;   // stopping and nothing waits
            }
            ige_op keep = nullptr;
            if (crc == IGE_OK) {
                run(grp, wctx, w, keep);
            } else {
                for (auto *r : grp) {
                    r->rc = crc;
                    r->err = "worker context creation failed";
                }
            }
            // keep the operator resident if the solve went through, else free it
            const bool healthy = keep && (grp[0]->rc == IGE_OK || grp[0]->rc == IGE_ENOTCONV);
            size_t bytes = 0;
            if (healthy) {
                ige_op_info_t info{};
                if (ige_op_info(keep, &info) == IGE_OK) bytes = (size_t)info.device_bytes;
            }
            ige_op freed = nullptr;
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= held;
                Resident &R = resident[w];
                if (healthy && !stop) {
                    R.op = keep;
                    R.geom = grp[0]->geom;
                    R.prm = grp[0]->prm;
                    R.bytes = bytes;
                    in_use += bytes;
                } else {
                    if (R.op == keep) R = Resident{};
                    freed = keep;
                }
                const double t = now();
                for (auto *r : grp) {
                    r->t_done = t;
                    r->state = 2;
                }
            }
            if (freed) ige_op_destroy(freed);
            cv_done.notify_all();
            cv_work.notify_all();
        }
        ige_op last = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (resident[w].op) {
                in_use -= resident[w].bytes;
                last = resident[w].op;
                resident[w] = Resident{};
            }
        }
        if (last) ige_op_destroy(last);
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
    st->merged = r.merged;
    st->reused = r.reused ? 1 : 0;
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
        srv->resident.resize(n_workers);
        ige_srv_s *s = srv.get();
        for (int i = 0; i < n_workers; ++i) s->workers.emplace_back([s, i] { s->worker_main(i); });
        ctx->users++;
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
        IGE_REQUIRE(prm->kind == IGE_OP_EFIE, "serving solves plane-wave scattering with the EFIE operator only");
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
        int mm = kMergeDefault;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            mm = srv->max_merge;
        }
        r->footprint = ige::planned_device_bytes(planned, opts->restart, n_waves, opts);
        r->fp_merged = ige::planned_device_bytes(planned, opts->restart, std::max(n_waves, mm), opts);
        r->fp_operator = ige::planned_device_bytes(planned, 0, 1, nullptr);
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
        srv->cv_work.notify_all();
    });
}

int ige_srv_set_merge(ige_srv srv, int max_waves)
{
    return srv_guard([&] {
        IGE_REQUIRE(srv, "null server");
        IGE_REQUIRE(max_waves >= 1 && max_waves <= 4096, "max_waves must be 1..4096");
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->max_merge = max_waves;
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
        srv->parent->users--;
        delete srv;
    });
}

}  // extern "C"
