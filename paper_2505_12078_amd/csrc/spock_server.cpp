// Served form: a continuous-batching request loop for MPC solves.
//
// Trees (problem data) are registered once; requests (tree, x0) arrive at any
// time from any thread.  A worker thread owns the device:
//  - admission: a request starts when its tree has no request in flight and
//    the tree is resident on the device, or can be made resident within the
//    HBM budget (footprint known before allocation; idle trees are evicted
//    least recently used first);
//  - every resident tree keeps its offline factors and its last iterate, so
//    the next request of a tree warm-starts from it (with its new x0);
//  - all requests in flight advance together: one batched chunk of
//    check_every CP steps per tick over every resident tree, with the trees
//    that have nothing to do switched off by their active flag; requests that
//    arrive meanwhile join at the next tick;
//  - mixed precision: float32 chunks, then a float64 check step, float64
//    chunks if the check fails (the same sequence as spock_solve, so a
//    request's result is the one it gets alone).

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "spock_internal.h"

namespace {

struct SrvTree {
    int64_t id = 0;
    int n = 0, nx = 0, nu = 0, n_nl = 0;
    std::vector<int32_t> parent;
    std::vector<double> prob, A, B, c, Q, R, QN, xlo, xhi, ulo, uhi, xNlo, xNhi, gamma, q, r, qN, Qe, Re, QNl, Qd, Rd, QNd, G, glo, ghi, GN, gNlo, gNhi;
    std::vector<double> rE, rF, rb;  // general coherent risks (empty: AV@R)
    std::vector<int32_t> rny, rnnu, rcone;
    double x_ball = 0, xN_ball = 0;
    size_t footprint = 0;
    spock_problem* p = nullptr;  // resident when non-null
    bool busy = false;           // a request of this tree is queued-in-flight
    bool has_iterate = false;    // a warm start is available
    double last_used = 0;

    spock_problem_desc desc() const {
        spock_problem_desc d{};
        d.n_nodes = n;
        d.parent = parent.data();
        d.cond_prob = prob.data();
        d.nx = nx;
        d.nu = nu;
        d.A = A.data();
        d.B = B.data();
        d.c = c.empty() ? nullptr : c.data();
        d.Q_diag = Q.empty() ? nullptr : Q.data();
        d.R_diag = R.empty() ? nullptr : R.data();
        d.QN_diag = QN.empty() ? nullptr : QN.data();
        d.Q_edge = Qe.empty() ? nullptr : Qe.data();
        d.R_edge = Re.empty() ? nullptr : Re.data();
        d.QN_leaf = QNl.empty() ? nullptr : QNl.data();
        d.Q_dense = Qd.empty() ? nullptr : Qd.data();
        d.R_dense = Rd.empty() ? nullptr : Rd.data();
        d.QN_dense = QNd.empty() ? nullptr : QNd.data();
        d.n_con = (int32_t)glo.size();
        d.Gamma = G.empty() ? nullptr : G.data();
        d.con_lo = glo.empty() ? nullptr : glo.data();
        d.con_hi = ghi.empty() ? nullptr : ghi.data();
        d.n_conN = (int32_t)gNlo.size();
        d.GammaN = GN.empty() ? nullptr : GN.data();
        d.conN_lo = gNlo.empty() ? nullptr : gNlo.data();
        d.conN_hi = gNhi.empty() ? nullptr : gNhi.data();
        d.x_lo = xlo.empty() ? nullptr : xlo.data();
        d.x_hi = xhi.empty() ? nullptr : xhi.data();
        d.u_lo = ulo.empty() ? nullptr : ulo.data();
        d.u_hi = uhi.empty() ? nullptr : uhi.data();
        d.xN_lo = xNlo.empty() ? nullptr : xNlo.data();
        d.xN_hi = xNhi.empty() ? nullptr : xNhi.data();
        d.x_ball = x_ball;
        d.xN_ball = xN_ball;
        d.gamma = gamma.empty() ? nullptr : gamma.data();
        d.risk_ny = rny.empty() ? nullptr : rny.data();
        d.risk_nnu = rnnu.empty() ? nullptr : rnnu.data();
        d.risk_E = rE.empty() ? nullptr : rE.data();
        d.risk_F = rF.empty() ? nullptr : rF.data();
        d.risk_b = rb.empty() ? nullptr : rb.data();
        d.risk_cone = rcone.empty() ? nullptr : rcone.data();
        d.q = q.empty() ? nullptr : q.data();
        d.r = r.empty() ? nullptr : r.data();
        d.qN = qN.empty() ? nullptr : qN.data();
        return d;
    }
};

struct SrvReq {
    uint64_t id = 0;
    int64_t tree = 0;
    std::vector<double> x0;
    double t_submit = 0, t_admit = 0;
};

struct Flight {
    SrvReq req;
    Member m;
    int phase = 0;  // 0: float32 chunks, 1: float64 chunks
    int warm = 0;
};

}  // namespace

struct spock_server {
    size_t budget = 0, used = 0;
    spock_settings set{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<SrvReq> pending;
    std::vector<spock_result> done;
    std::map<int64_t, SrvTree> trees;
    int64_t next_tree = 1;
    size_t inflight = 0;  // admitted and not finished
    std::thread worker;
    bool stop = false;
    std::string error;
    spock_server_stats stats{};
    // set-up thread: trees made resident off the worker's critical path
    std::thread setup;
    std::deque<int64_t> setup_jobs;              // trees to create (budget reserved)
    std::deque<std::pair<int64_t, spock_problem*>> setup_done;  // created (or null on failure)
    std::map<int64_t, SrvReq> waiting;           // admitted requests whose tree is being set up
    size_t reserved = 0;                         // budget of trees being set up
    // worker-owned
    spock_batch* batch = nullptr;
    std::vector<int64_t> members;
    bool dirty = true;
    std::map<int64_t, Flight> flights;
};

namespace {

// Lookup under the lock (map nodes stay put when other trees are added).
SrvTree& tree_ref(spock_server* s, int64_t id) {
    std::lock_guard<std::mutex> g(s->mu);
    return s->trees.at(id);
}

void finish(spock_server* s, Flight& f, int32_t status, double t) {
    spock_result r{};
    r.req_id = f.req.id;
    r.tree_id = f.req.tree;
    r.status = status;
    r.warm = f.warm;
    r.info.iters = f.m.iters;
    r.info.iters_fp32 = f.m.iters32;
    r.info.rel_res = f.m.rel;
    r.info.xi1_inf = f.m.x1;
    r.info.xi2_inf = f.m.x2;
    r.info.status = status;
    r.info.refined = f.m.refined;
    r.t_submit = f.req.t_submit;
    r.t_admit = f.req.t_admit;
    r.t_done = t;
    SrvTree& T = tree_ref(s, f.req.tree);
    if (T.p && status != SPOCK_E_INFEASIBLE_X0 && status != SPOCK_E_HIP) {
        double s0 = 0;
        if (T.p->cur == SPOCK_FP64) {
            (void)hipMemcpy(&s0, T.p->s64.h.z[T.p->s64.par], 8, hipMemcpyDeviceToHost);
        } else {
            float v = 0;
            (void)hipMemcpy(&v, T.p->s32.h.z[T.p->s32.par], 4, hipMemcpyDeviceToHost);
            s0 = v;
        }
        r.info.s0 = s0;
        r.info.precision_used = T.p->cur;
        r.info.t_setup_s = T.p->t_setup;
        T.has_iterate = true;
        T.p->solved = true;
    }
    r.info.t_solve_s = t - f.req.t_admit;
    std::lock_guard<std::mutex> g(s->mu);
    T.busy = false;
    T.last_used = t;
    s->done.push_back(r);
    s->inflight--;
    s->stats.completed++;
    s->cv.notify_all();
}

// Admit what fits; returns the requests to start (trees made resident by the caller).
std::vector<SrvReq> admit(spock_server* s, std::vector<int64_t>& to_create, std::vector<int64_t>& to_evict) {
    std::vector<SrvReq> out;
    size_t used = s->used + s->reserved;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        SrvTree& T = s->trees.at(it->tree);
        if (T.busy) {
            ++it;
            continue;
        }
        if (!T.p) {
            if (used + T.footprint > s->budget) {
                // evict idle resident trees, least recently used first; the
                // victims are chosen first and evicted only if the tree then
                // fits, so a request that cannot start destroys nothing
                std::vector<SrvTree*> idle;
                for (auto& kv : s->trees)
                    if (kv.second.p && !kv.second.busy &&
                        std::find(to_evict.begin(), to_evict.end(), kv.first) == to_evict.end())
                        idle.push_back(&kv.second);
                std::sort(idle.begin(), idle.end(), [](SrvTree* a, SrvTree* b) { return a->last_used < b->last_used; });
                std::vector<SrvTree*> victims;
                size_t freed = 0;
                for (SrvTree* v : idle) {
                    if (used - freed + T.footprint <= s->budget) break;
                    victims.push_back(v);
                    freed += v->footprint;
                }
                if (used - freed + T.footprint > s->budget) {
                    ++it;
                    continue;
                }
                for (SrvTree* v : victims) {
                    to_evict.push_back(v->id);
                    v->busy = true;  // nobody touches it until it is gone
                }
                used -= freed;
            }
            used += T.footprint;
            to_create.push_back(T.id);
        }
        T.busy = true;
        it->t_admit = now_s();
        out.push_back(*it);
        it = s->pending.erase(it);
    }
    return out;
}

int32_t start_flight(spock_server* s, SrvReq& rq) {
    SrvTree& T = tree_ref(s, rq.tree);
    Flight f;
    f.req = rq;
    f.warm = T.has_iterate ? 1 : 0;
    spock_problem* p = T.p;
    int32_t r = set_x0_device(p, rq.x0.data(), true);
    if (r) {
        finish(s, f, r, now_s());
        return SPOCK_OK;
    }
    long long taken = 0;
    double a1 = 0, a2 = 0;
    r = ensure_ref(p, f.warm != 0, &taken, &a1, &a2);
    const int prec = s->set.precision;
    if (!r) r = move_iterate(p, prec == SPOCK_FP64 ? SPOCK_FP64 : SPOCK_FP32);
    if (!r) r = normalize_parity(p);
    if (!r && hipStreamSynchronize(p->stream) != hipSuccess) r = fail(SPOCK_E_HIP, "sync");
    if (r) return r;
    f.m.iters = taken;
    if (taken) {
        f.m.x1 = a1;
        f.m.x2 = a2;
        f.m.rel = rel_of(a1, a2, std::max(1.0, std::max(a1, a2)));
    }
    f.m.live = f.m.iters < s->set.max_iters;
    f.phase = prec == SPOCK_FP64 ? 1 : 0;
    if (!f.m.live) {
        finish(s, f, SPOCK_E_NOT_CONVERGED, now_s());
        return SPOCK_OK;
    }
    s->flights[rq.tree] = f;
    return SPOCK_OK;
}

int32_t rebuild_batch(spock_server* s) {
    if (s->batch) {
        spock_batch_destroy(s->batch);
        s->batch = nullptr;
    }
    s->members.clear();
    std::vector<spock_problem*> ps;
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (auto& kv : s->trees)
            if (kv.second.p) {
                s->members.push_back(kv.first);
                ps.push_back(kv.second.p);
            }
    }
    s->dirty = false;
    if (ps.empty()) return SPOCK_OK;
    return spock_batch_create(ps.data(), (int32_t)ps.size(), &s->set, &s->batch);
}

// One tick: a float32 chunk for the flights in their float32 phase and a
// float64 chunk for the others, then phase changes and completions.
int32_t tick(spock_server* s) {
    if (s->flights.empty() || !s->batch) return SPOCK_OK;
    const int n = (int)s->members.size();
    for (int phase = 0; phase < 2; ++phase) {
        std::vector<Member> m(n);
        bool any = false;
        for (int k = 0; k < n; ++k) {
            auto it = s->flights.find(s->members[k]);
            if (it != s->flights.end() && it->second.phase == phase && it->second.m.live) {
                m[k] = it->second.m;
                any = true;
            }
        }
        if (!any) continue;
        int32_t r = phase == 0 ? batch_tick<float>(s->batch, m, s->set.precision == SPOCK_MIXED)
                               : batch_tick<double>(s->batch, m, false);
        if (r) return r;
        for (int k = 0; k < n; ++k) {
            auto it = s->flights.find(s->members[k]);
            if (it != s->flights.end() && it->second.phase == phase && it->second.m.live) it->second.m = m[k];
        }
    }
    // transitions
    const double t = now_s();
    for (auto it = s->flights.begin(); it != s->flights.end();) {
        Flight& f = it->second;
        if (f.m.live) {
            ++it;
            continue;
        }
        spock_problem* p = tree_ref(s, f.req.tree).p;
        bool complete = true;
        if (f.phase == 0 && s->set.precision == SPOCK_MIXED &&
            (f.m.status == SPOCK_OK || f.m.status == SPOCK_E_NOT_CONVERGED)) {
            // float64 check of the float32 iterate
            double a1, a2;
            p->cur = SPOCK_FP32;
            p->s32.par = 0;
            int32_t r = move_iterate(p, SPOCK_FP64);
            if (!r) r = step<double>(p, 1);
            if (!r) r = read_res(p, &a1, &a2);
            if (!r) r = normalize_parity(p);
            if (!r && hipStreamSynchronize(p->stream) != hipSuccess) r = fail(SPOCK_E_HIP, "sync");
            if (r) return r;
            f.m.iters += 1;
            f.m.x1 = a1;
            f.m.x2 = a2;
            f.m.rel = rel_of(a1, a2, std::max(1.0, std::max(p->xi_ref[0], p->xi_ref[1])));
            if (f.m.rel <= s->set.eps) {
                f.m.status = SPOCK_OK;
            } else if (f.m.iters < s->set.max_iters) {
                f.m.refined = 1;
                f.m.live = true;
                f.phase = 1;
                complete = false;
            } else {
                f.m.status = SPOCK_E_NOT_CONVERGED;
            }
        } else if (f.phase == 0) {
            p->cur = SPOCK_FP32;
            p->s32.par = 0;
        } else {
            p->cur = SPOCK_FP64;
            p->s64.par = 0;
        }
        if (complete) {
            finish(s, f, f.m.status, t);
            it = s->flights.erase(it);
        } else {
            ++it;
        }
    }
    return SPOCK_OK;
}

void setup_main(spock_server* s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        int64_t id;
        spock_problem_desc d;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv.wait(g, [&] { return s->stop || !s->setup_jobs.empty(); });
            if (s->stop) return;
            id = s->setup_jobs.front();
            s->setup_jobs.pop_front();
            d = s->trees.at(id).desc();
        }
        spock_problem* p = nullptr;
        if (spock_problem_create(&d, &s->set, nullptr, 0, nullptr, &p) != SPOCK_OK) p = nullptr;
        std::lock_guard<std::mutex> g(s->mu);
        s->setup_done.emplace_back(id, p);
        if (p) s->stats.created++;
        s->cv.notify_all();
    }
}

void worker_main(spock_server* s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<int64_t> to_create, to_evict;
        std::vector<SrvReq> start;
        std::deque<std::pair<int64_t, spock_problem*>> ready;
        {
            std::unique_lock<std::mutex> g(s->mu);
            if (s->stop) break;
            std::vector<SrvReq> adm = admit(s, to_create, to_evict);
            for (auto& rq : adm) {
                if (std::find(to_create.begin(), to_create.end(), rq.tree) != to_create.end())
                    s->waiting[rq.tree] = rq;  // starts when its tree is set up
                else
                    start.push_back(rq);
            }
            ready.swap(s->setup_done);
            if (start.empty() && ready.empty() && s->flights.empty() && to_evict.empty()) {
                if (to_create.empty()) {
                    s->cv.wait_for(g, std::chrono::milliseconds(20));
                    continue;
                }
            }
        }
        int32_t r = SPOCK_OK;
        for (int64_t id : to_evict) {
            SrvTree& T = tree_ref(s, id);
            spock_problem_destroy(T.p);
            T.p = nullptr;
            T.has_iterate = false;
            s->used -= T.footprint;
            s->dirty = true;
            std::lock_guard<std::mutex> g(s->mu);
            T.busy = false;
            s->stats.evicted++;
        }
        if (!to_create.empty()) {
            std::lock_guard<std::mutex> g(s->mu);
            for (int64_t id : to_create) {
                s->reserved += s->trees.at(id).footprint;
                s->setup_jobs.push_back(id);
            }
            s->cv.notify_all();
        }
        for (auto& rd : ready) {
            SrvTree& T = tree_ref(s, rd.first);
            SrvReq rq;
            {
                std::lock_guard<std::mutex> g(s->mu);
                s->reserved -= T.footprint;
                rq = s->waiting.at(rd.first);
                s->waiting.erase(rd.first);
            }
            if (!rd.second) {  // set-up failed: report and free the tree
                Flight f;
                f.req = rq;
                finish(s, f, SPOCK_E_NOMEM, now_s());
                continue;
            }
            T.p = rd.second;
            s->used += T.footprint;
            s->dirty = true;
            start.push_back(rq);
        }
        for (auto& rq : start) {
            if (r) break;
            r = start_flight(s, rq);
        }
        if (!r && s->dirty) r = rebuild_batch(s);
        if (!r) r = tick(s);
        if (r) {
            std::lock_guard<std::mutex> g(s->mu);
            s->error = g_err;
            s->stop = true;
            s->cv.notify_all();
            break;
        }
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stats.resident_bytes = s->used;
            s->stats.ticks++;
        }
    }
}

}  // namespace

extern "C" {

int32_t spock_server_create(size_t budget, const spock_settings* set, spock_server** out) {
    if (!out || !set || budget == 0) return fail(SPOCK_E_INVALID, "bad server arguments");
    if (set->method != SPOCK_CP) return fail(SPOCK_E_INVALID, "the served form runs plain CP iterations");
    if (set->check_every < 2 || (set->check_every & 1) || !(set->eps > 0) || set->max_iters < 1)
        return fail(SPOCK_E_INVALID, "bad server settings");
    spock_server* s = new spock_server();
    s->budget = budget;
    s->set = *set;
    (void)hipGetDevice(&s->device);
    s->worker = std::thread(worker_main, s);
    s->setup = std::thread(setup_main, s);
    *out = s;
    return SPOCK_OK;
}

int32_t spock_server_add_tree(spock_server* s, const spock_problem_desc* d, int64_t* tree_id) {
    if (!s || !d || !tree_id) return fail(SPOCK_E_INVALID, "null argument");
    size_t fp = 0;
    int32_t r = spock_problem_footprint(d, &s->set, &fp);
    if (r) return r;
    if (fp > s->budget) return fail(SPOCK_E_CAPACITY, "tree footprint exceeds the whole device budget");
    SrvTree T;
    T.n = d->n_nodes;
    T.nx = d->nx;
    T.nu = d->nu;
    const size_t n = T.n, nx = T.nx, nu = T.nu;
    T.parent.assign(d->parent, d->parent + n);
    for (size_t j = 0; j < n; ++j) T.n_nl = std::max<int>(T.n_nl, d->parent[j] + 1);
    T.prob.assign(d->cond_prob, d->cond_prob + n);
    T.A.assign(d->A, d->A + n * nx * nx);
    T.B.assign(d->B, d->B + n * nx * nu);
    if (d->c) T.c.assign(d->c, d->c + n * nx);
    if (d->q) T.q.assign(d->q, d->q + n * nx);
    if (d->r) T.r.assign(d->r, d->r + n * nu);
    if (d->qN) T.qN.assign(d->qN, d->qN + n * nx);
    if (d->Q_diag) T.Q.assign(d->Q_diag, d->Q_diag + nx);
    if (d->R_diag) T.R.assign(d->R_diag, d->R_diag + nu);
    if (d->QN_diag) T.QN.assign(d->QN_diag, d->QN_diag + nx);
    if (d->Q_edge) T.Qe.assign(d->Q_edge, d->Q_edge + n * nx);
    if (d->R_edge) T.Re.assign(d->R_edge, d->R_edge + n * nu);
    if (d->QN_leaf) T.QNl.assign(d->QN_leaf, d->QN_leaf + n * nx);
    if (d->Q_dense) T.Qd.assign(d->Q_dense, d->Q_dense + n * nx * nx);
    if (d->R_dense) T.Rd.assign(d->R_dense, d->R_dense + n * nu * nu);
    if (d->QN_dense) T.QNd.assign(d->QN_dense, d->QN_dense + n * nx * nx);
    if (d->Gamma) {
        const size_t nr = (size_t)d->n_con;
        T.G.assign(d->Gamma, d->Gamma + nr * (nx + nu));
        T.glo.assign(d->con_lo, d->con_lo + nr);
        T.ghi.assign(d->con_hi, d->con_hi + nr);
    }
    if (d->GammaN) {
        const size_t nr = (size_t)d->n_conN;
        T.GN.assign(d->GammaN, d->GammaN + nr * nx);
        T.gNlo.assign(d->conN_lo, d->conN_lo + nr);
        T.gNhi.assign(d->conN_hi, d->conN_hi + nr);
    }
    // the box of the non-leaf (leaf) nodes may be absent when general rows replace it
    if (d->x_lo) T.xlo.assign(d->x_lo, d->x_lo + nx);
    if (d->x_hi) T.xhi.assign(d->x_hi, d->x_hi + nx);
    if (d->u_lo) T.ulo.assign(d->u_lo, d->u_lo + nu);
    if (d->u_hi) T.uhi.assign(d->u_hi, d->u_hi + nu);
    if (d->xN_lo) T.xNlo.assign(d->xN_lo, d->xN_lo + nx);
    if (d->xN_hi) T.xNhi.assign(d->xN_hi, d->xN_hi + nx);
    T.x_ball = d->x_ball;
    T.xN_ball = d->xN_ball;
    T.footprint = fp;
    // non-leaf count from the validated layout: every parent index is a non-leaf node
    std::vector<char> nonleaf(n, 0);
    for (size_t j = 1; j < n; ++j) nonleaf[d->parent[j]] = 1;
    T.n_nl = (int)std::count(nonleaf.begin(), nonleaf.end(), 1);
    if (d->gamma) T.gamma.assign(d->gamma, d->gamma + T.n_nl);
    if (d->risk_ny) {  // sizes from the validated layout: children per non-leaf node
        std::vector<long long> kids(T.n_nl, 0);
        for (size_t j = 1; j < n; ++j) kids[d->parent[j]]++;
        long long tE = 0, tF = 0, tb = 0;
        for (int i = 0; i < T.n_nl; ++i) {
            tE += (long long)d->risk_ny[i] * kids[i];
            tF += (long long)d->risk_ny[i] * d->risk_nnu[i];
            tb += d->risk_ny[i];
        }
        T.rny.assign(d->risk_ny, d->risk_ny + T.n_nl);
        T.rnnu.assign(d->risk_nnu, d->risk_nnu + T.n_nl);
        T.rE.assign(d->risk_E, d->risk_E + tE);
        if (tF > 0) T.rF.assign(d->risk_F, d->risk_F + tF);
        T.rb.assign(d->risk_b, d->risk_b + tb);
        T.rcone.assign(d->risk_cone, d->risk_cone + tb);
    }
    std::lock_guard<std::mutex> g(s->mu);
    T.id = s->next_tree++;
    *tree_id = T.id;
    s->trees[T.id] = std::move(T);
    return SPOCK_OK;
}

int32_t spock_server_submit(spock_server* s, int64_t tree_id, const double* x0, uint64_t req_id) {
    if (!s || !x0) return fail(SPOCK_E_INVALID, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(SPOCK_E_HIP, "server stopped: " + s->error);
    auto it = s->trees.find(tree_id);
    if (it == s->trees.end()) return fail(SPOCK_E_INVALID, "unknown tree");
    SrvReq rq;
    rq.id = req_id;
    rq.tree = tree_id;
    rq.x0.assign(x0, x0 + it->second.nx);
    rq.t_submit = now_s();
    s->pending.push_back(std::move(rq));
    s->inflight++;
    s->stats.submitted++;
    s->cv.notify_all();
    return SPOCK_OK;
}

int32_t spock_server_poll(spock_server* s, spock_result* out, int32_t max, int32_t* n_out) {
    if (!s || !n_out || (max > 0 && !out)) return fail(SPOCK_E_INVALID, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    const int32_t k = (int32_t)std::min<size_t>(max > 0 ? (size_t)max : 0, s->done.size());
    for (int32_t i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n_out = k;
    if (s->stop && !s->error.empty()) return fail(SPOCK_E_HIP, "server stopped: " + s->error);
    return SPOCK_OK;
}

int32_t spock_server_wait_idle(spock_server* s, double timeout_s) {
    if (!s) return fail(SPOCK_E_INVALID, "null server");
    std::unique_lock<std::mutex> g(s->mu);
    const bool ok = s->cv.wait_for(g, std::chrono::duration<double>(timeout_s),
                                   [&] { return s->inflight == 0 || s->stop; });
    if (s->stop && !s->error.empty()) return fail(SPOCK_E_HIP, "server stopped: " + s->error);
    return ok ? SPOCK_OK : fail(SPOCK_E_NOT_CONVERGED, "server not idle before the timeout");
}

int32_t spock_server_get_stats(spock_server* s, spock_server_stats* out) {
    if (!s || !out) return fail(SPOCK_E_INVALID, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->budget_bytes = s->budget;
    out->pending = s->pending.size();
    out->in_flight = s->inflight - s->pending.size();
    return SPOCK_OK;
}

int32_t spock_server_solution(spock_server* s, int64_t tree_id, double* x, double* u, double* s0) {
    if (!s) return fail(SPOCK_E_INVALID, "null server");
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->trees.find(tree_id);
    if (it == s->trees.end() || !it->second.p) return fail(SPOCK_E_INVALID, "tree not resident");
    if (it->second.busy) return fail(SPOCK_E_INVALID, "tree has a request in flight");
    return spock_get_solution(it->second.p, x, u, s0);
}

double spock_now(void) { return now_s(); }

int32_t spock_server_destroy(spock_server* s) {
    if (!s) return SPOCK_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (s->setup.joinable()) s->setup.join();
    for (auto& rd : s->setup_done)
        if (rd.second) spock_problem_destroy(rd.second);
    if (s->batch) spock_batch_destroy(s->batch);
    for (auto& kv : s->trees)
        if (kv.second.p) spock_problem_destroy(kv.second.p);
    delete s;
    return SPOCK_OK;
}

}  // extern "C"
