// Batched form: many independent scenario trees advanced by the same four
// launches per CP step as one tree.  Each member keeps its own workspace; the
// batch holds copies of the members' descriptors whose residual slots and
// "active" flags point into batch-owned arrays, two problem-major
// task tables (one sweep task per leaf and one node task per node of every
// member).
// Members that converge are switched off through their active flag, so a
// captured graph of `check_every` steps is replayed unchanged until every
// member is done.

#include <algorithm>
#include <cmath>
#include <cstring>

#include "spock_internal.h"

namespace {


template <typename real>
ProbDev<real>* dev_of(spock_batch* b);
template <>
ProbDev<double>* dev_of<double>(spock_batch* b) { return b->d64; }
template <>
ProbDev<float>* dev_of<float>(spock_batch* b) { return b->d32; }
template <typename real>
spk::LaunchCfg& cfg_of(spock_batch* b) { return sizeof(real) == 8 ? b->cfg64 : b->cfg32; }

// The batch's launch configuration: LDS sizes and tile classes large enough
// for every member, the node workgroup lowered until its LDS fits 64 KiB.
template <typename real>
spk::LaunchCfg batch_cfg(const spock_batch* b, int node_wg) {
    spk::LaunchCfg c{};
    int cst = 0;
    for (auto* p : b->probs) {
        const spk::LaunchCfg m = make_cfg<real>(p, 64);
        c.wave_elems = std::max(c.wave_elems, m.wave_elems);
        c.sweep_lds = std::max(c.sweep_lds, m.sweep_lds);
        for (int q = 0; q < 4; ++q) c.cls[q] = std::max(c.cls[q], m.cls[q]);
        c.dense = std::max(c.dense, m.dense);
        cst = std::max(cst, spk::consts_elems(p->nx, p->nu));
    }
    auto lds = [&](int wg) { return (cst + (wg / 64) * c.wave_elems) * (int)sizeof(real); };
    while (node_wg > 64 && lds(node_wg) > 64 * 1024) node_wg /= 2;
    c.leaf_tasks = b->tasks;
    c.n_leaf_tasks = b->n_tasks;
    c.node_tasks = b->ntasks;
    c.node_info = b->ninfo;
    c.n_node_tasks = b->n_ntasks;
    c.node_wg = node_wg;
    c.node_lds = lds(node_wg);
    return c;
}

int32_t upload_active(spock_batch* b, const std::vector<Member>* m) {
    for (int k = 0; k < b->n; ++k) b->h_active[k] = m ? (int)(*m)[k].live : 1;
    HIP_TRY(hipMemcpyAsync(b->active, b->h_active.data(), b->n * sizeof(int), hipMemcpyHostToDevice, b->stream));
    return SPOCK_OK;
}

template <typename real>
int32_t batch_steps(spock_batch* b, int steps, bool check_last) {
    for (int k = 0; k < steps; ++k) {
        // every member sits at copy 0 before a batched chunk; parity follows k
        HIP_TRY(spk::launch_step<real>(dev_of<real>(b), cfg_of<real>(b), k & 1, check_last && k == steps - 1,
                                       b->stream));
    }
    return SPOCK_OK;
}

template <typename real>
int32_t batch_chunk(spock_batch* b, int steps) {
    const int gi = sizeof(real) == 8 ? 0 : 1;
    if (!b->set.use_graph) return batch_steps<real>(b, steps, true);
    if (b->graph_steps[gi] != steps && b->graph[gi]) {
        (void)hipGraphExecDestroy(b->graph[gi]);
        b->graph[gi] = nullptr;
    }
    if (!b->graph[gi]) {
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        hipGraph_t g;
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        int32_t r = batch_steps<real>(b, steps, true);
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (r) return r;
        if (e != hipSuccess) return fail(SPOCK_E_HIP, std::string("capture: ") + hipGetErrorString(e));
        HIP_TRY(hipGraphInstantiate(&b->graph[gi], g, nullptr, nullptr, 0));
        HIP_TRY(hipGraphDestroy(g));
        b->graph_steps[gi] = steps;
    }
    HIP_TRY(hipGraphLaunch(b->graph[gi], b->stream));
    return SPOCK_OK;
}

int32_t read_all(spock_batch* b) {
    HIP_TRY(hipMemcpyAsync(b->h_res, b->res, 2 * spk::kResSlots * b->n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SPOCK_OK;
}

}  // namespace

// One chunk of check_every steps for the live members; updates their state.
template <typename real>
int32_t batch_tick(spock_batch* b, std::vector<Member>& m, bool stall_exit) {
    const int ce = b->set.check_every;
    {
        int32_t r = upload_active(b, &m);
        if (!r) r = batch_chunk<real>(b, ce);
        if (!r) r = read_all(b);
        if (r) return r;
        for (int k = 0; k < b->n; ++k) {
            Member& x = m[k];
            if (!x.live) continue;
            spock_problem* p = b->probs[k];
            x.iters += ce;
            if (sizeof(real) == 4) x.iters32 += ce;
            res_reduce(b->h_res + 2 * spk::kResSlots * k, &x.x1, &x.x2);
            x.rel = rel_of(x.x1, x.x2, std::max(1.0, std::max(p->xi_ref[0], p->xi_ref[1])));
            if (!std::isfinite(x.rel)) {
                x.status = SPOCK_E_DIVERGED;
                x.live = false;
            } else if (x.rel <= b->set.eps) {
                x.status = SPOCK_OK;
                x.live = false;
            } else if (x.iters >= b->set.max_iters) {
                x.status = SPOCK_E_NOT_CONVERGED;
                x.live = false;
            } else if (stall_exit) {
                ++x.checks;
                if (x.rel < 0.99 * x.best) {
                    x.best = x.rel;
                    x.no_gain = 0;
                } else if (++x.no_gain >= std::max(50, x.checks / 2)) {
                    x.status = SPOCK_E_NOT_CONVERGED;
                    x.live = false;
                }
            }
        }
    }
    return SPOCK_OK;
}
template int32_t batch_tick<double>(spock_batch*, std::vector<Member>&, bool);
template int32_t batch_tick<float>(spock_batch*, std::vector<Member>&, bool);

// Iterate every live member in one precision until it converges, stalls
// (float32 only) or spends its budget.
template <typename real>
static int32_t batch_phase(spock_batch* b, std::vector<Member>& m, bool stall_exit) {
    for (;;) {
        bool any = false;
        for (auto& x : m) any = any || x.live;
        if (!any) return SPOCK_OK;
        int32_t r = batch_tick<real>(b, m, stall_exit);
        if (r) return r;
    }
}

extern "C" {

int32_t spock_batch_create(spock_problem* const* probs, int32_t n, const spock_settings* s, spock_batch** out) {
    if (!out || !probs || n < 1 || !s) return fail(SPOCK_E_INVALID, "bad batch arguments");
    *out = nullptr;
    if (s->method != SPOCK_CP) return fail(SPOCK_E_INVALID, "the batched form runs plain CP iterations");
    if (s->check_every < 2 || (s->check_every & 1) || !(s->eps > 0) || s->max_iters < 1 ||
        s->precision < SPOCK_FP64 || s->precision > SPOCK_FP32)
        return fail(SPOCK_E_INVALID, "bad batch settings");
    spock_batch* b = new spock_batch();
    b->n = n;
    b->set = *s;
    b->probs.assign(probs, probs + n);
    for (int k = 0; k < n; ++k) {
        if (!probs[k]) {
            delete b;
            return fail(SPOCK_E_INVALID, "null problem in batch");
        }
        b->n_tasks += probs[k]->n_leaf;
        b->n_ntasks += probs[k]->n_ntasks;
        HIP_TRY(hipStreamSynchronize(probs[k]->stream));
        for (int q = 0; q < 2; ++q) {
            double kb[4];
            step_bytes_of(probs[k], q == 0 ? 8 : 4, kb);
            for (int ph = 0; ph < 4; ++ph) b->bytes_k[q][ph] += kb[ph];
        }
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        size_t o = off;
        off += std::max<size_t>(bytes, 1);
        return o;
    };
    const size_t o64 = take(sizeof(ProbDev<double>) * n), o32 = take(sizeof(ProbDev<float>) * n);
    const size_t ot = take(sizeof(int2) * b->n_tasks), oa = take(sizeof(int) * n);
    const size_t ont = take(sizeof(int2) * b->n_ntasks), oni = take(sizeof(int4) * b->n_ntasks);
    const size_t orr = take(sizeof(unsigned long long) * 2 * spk::kResSlots * n);
    b->bytes = off + 256;
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    hipError_t e = hipMalloc(&b->base, b->bytes);
    if (e != hipSuccess) {
        delete b;
        return fail(SPOCK_E_NOMEM, std::string("batch hipMalloc: ") + hipGetErrorString(e));
    }
    char* base = (char*)b->base;
    b->d64 = (ProbDev<double>*)(base + o64);
    b->d32 = (ProbDev<float>*)(base + o32);
    b->tasks = (int2*)(base + ot);
    b->ntasks = (int2*)(base + ont);
    b->ninfo = (int4*)(base + oni);
    b->active = (int*)(base + oa);
    b->res = (unsigned long long*)(base + orr);
    auto bail = [&](int32_t code, const std::string& msg) {
        spock_batch_destroy(b);
        return fail(code, msg);
    };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(SPOCK_E_HIP, "batch stream");
    if (hipHostMalloc((void**)&b->h_res, 2 * spk::kResSlots * n * sizeof(unsigned long long), 0) != hipSuccess)
        return bail(SPOCK_E_HIP, "batch pinned buffer");
    std::vector<ProbDev<double>> h64(n);
    std::vector<ProbDev<float>> h32(n);
    std::vector<int2> tasks, ntasks;
    std::vector<int4> ninfo;
    tasks.reserve(b->n_tasks);
    ntasks.reserve(b->n_ntasks);
    ninfo.reserve(b->n_ntasks);
    for (int k = 0; k < n; ++k) {
        h64[k] = probs[k]->s64.h;
        h32[k] = probs[k]->s32.h;
        h64[k].active = h32[k].active = b->active + k;
        h64[k].res = h32[k].res = b->res + 2 * spk::kResSlots * k;
        for (int l = 0; l < probs[k]->n_leaf; ++l) tasks.push_back(make_int2(k, l));
        const spock_problem* q = probs[k];
        for (int v = 0; v < q->n_ntasks; ++v) {
            ntasks.push_back(make_int2(k, v < q->n ? v : -1));
            if (v < q->n)
                ninfo.push_back(make_int4(q->n_ch[v] ? q->first_child[v] : 0, q->n_ch[v], v < q->n_nl ? q->y_off[v] : 0,
                                          q->parent[v]));
            else
                ninfo.push_back(make_int4(0, 0, 0, 0));
        }
    }
    b->cfg64 = batch_cfg<double>(b, spk::kDefaultWG);
    b->cfg32 = batch_cfg<float>(b, spk::kDefaultWG);
    b->h_active.assign(n, 1);
    e = hipMemcpy(b->d64, h64.data(), sizeof(ProbDev<double>) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d32, h32.data(), sizeof(ProbDev<float>) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->tasks, tasks.data(), sizeof(int2) * tasks.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->ntasks, ntasks.data(), sizeof(int2) * ntasks.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->ninfo, ninfo.data(), sizeof(int4) * ninfo.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->active, b->h_active.data(), sizeof(int) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->res, 0, sizeof(unsigned long long) * 2 * spk::kResSlots * n);
    if (e != hipSuccess) return bail(SPOCK_E_HIP, std::string("batch upload: ") + hipGetErrorString(e));
    *out = b;
    return SPOCK_OK;
}

int32_t spock_batch_destroy(spock_batch* b) {
    if (!b) return SPOCK_OK;
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& g : b->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (b->h_res) (void)hipHostFree(b->h_res);
    if (b->base) (void)hipFree(b->base);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return SPOCK_OK;
}

int32_t spock_batch_size(const spock_batch* b, int32_t* n_problems, int32_t* n_tasks, size_t* device_bytes) {
    if (!b) return fail(SPOCK_E_INVALID, "null batch");
    if (n_problems) *n_problems = b->n;
    if (n_tasks) *n_tasks = b->n_tasks;
    if (device_bytes) *device_bytes = b->bytes;
    return SPOCK_OK;
}

int32_t spock_batch_solve(spock_batch* b, const double* const* x0s, const int32_t* warm, spock_info* infos) {
    if (!b || !x0s || !infos) return fail(SPOCK_E_INVALID, "null batch argument");
    const double t0 = now_s();
    const int n = b->n;
    const int prec = b->set.precision;
    std::vector<Member> m(n);
    int32_t r = SPOCK_OK;
    // set-up: x0, cold starts, reference residuals, every member at copy 0 of
    // the phase precision
    for (int k = 0; k < n; ++k) {
        spock_problem* p = b->probs[k];
        std::memset(&infos[k], 0, sizeof(spock_info));
        const bool w = warm && warm[k];
        int32_t rk = set_x0_device(p, x0s[k], true);
        long long taken = 0;
        double a1, a2;
        if (!rk) rk = ensure_ref(p, w, &taken, &a1, &a2);
        if (!rk) {
            m[k].iters = taken;
            if (taken) {
                m[k].x1 = a1;
                m[k].x2 = a2;
                m[k].rel = std::max(a1, a2) / std::max(1.0, std::max(a1, a2));
            }
            rk = move_iterate(p, prec == SPOCK_FP64 ? SPOCK_FP64 : SPOCK_FP32);
        }
        if (!rk) rk = normalize_parity(p);
        if (!rk) rk = hipStreamSynchronize(p->stream) == hipSuccess ? SPOCK_OK : fail(SPOCK_E_HIP, "sync");
        if (rk) {
            m[k].status = rk;
            infos[k].status = rk;
            continue;
        }
        m[k].live = m[k].iters < b->set.max_iters;
    }
    if (prec == SPOCK_FP64) {
        r = batch_phase<double>(b, m, false);
    } else {
        r = batch_phase<float>(b, m, prec == SPOCK_MIXED);
        if (!r && prec == SPOCK_MIXED) {
            // float64 check of every float32 result; refine the ones that fail
            std::vector<Member> m2 = m;
            for (int k = 0; k < n; ++k) {
                m2[k].live = false;
                if (m[k].status != SPOCK_OK && m[k].status != SPOCK_E_NOT_CONVERGED) continue;
                spock_problem* p = b->probs[k];
                p->cur = SPOCK_FP32;
                p->s32.par = 0;
                double a1, a2;
                r = move_iterate(p, SPOCK_FP64);
                if (!r) r = step<double>(p, 1);
                if (!r) r = read_res(p, &a1, &a2);
                if (!r) r = normalize_parity(p);
                if (!r) r = hipStreamSynchronize(p->stream) == hipSuccess ? SPOCK_OK : fail(SPOCK_E_HIP, "sync");
                if (r) return r;
                m2[k].iters += 1;
                m2[k].x1 = a1;
                m2[k].x2 = a2;
                m2[k].rel = std::max(a1, a2) / std::max(1.0, std::max(p->xi_ref[0], p->xi_ref[1]));
                if (m2[k].rel <= b->set.eps) {
                    m2[k].status = SPOCK_OK;
                } else if (m2[k].iters < b->set.max_iters) {
                    m2[k].refined = 1;
                    m2[k].live = true;
                } else {
                    m2[k].status = SPOCK_E_NOT_CONVERGED;
                }
            }
            r = batch_phase<double>(b, m2, false);
            m.swap(m2);
        }
    }
    if (r) return r;
    // results
    for (int k = 0; k < n; ++k) {
        if (infos[k].status != SPOCK_OK && m[k].status != SPOCK_OK && m[k].iters == 0) continue;
        spock_problem* p = b->probs[k];
        if (prec == SPOCK_FP64 || prec == SPOCK_MIXED) {
            p->cur = SPOCK_FP64;
            p->s64.par = 0;
        } else {
            p->cur = SPOCK_FP32;
            p->s32.par = 0;
        }
        p->solved = true;
        double s0 = 0;
        if (p->cur == SPOCK_FP64) {
            HIP_TRY(hipMemcpy(&s0, p->s64.h.z[0], 8, hipMemcpyDeviceToHost));
        } else {
            float f;
            HIP_TRY(hipMemcpy(&f, p->s32.h.z[0], 4, hipMemcpyDeviceToHost));
            s0 = f;
        }
        infos[k].iters = m[k].iters;
        infos[k].iters_fp32 = m[k].iters32;
        infos[k].rel_res = m[k].rel;
        infos[k].xi1_inf = m[k].x1;
        infos[k].xi2_inf = m[k].x2;
        infos[k].s0 = s0;
        infos[k].status = m[k].status;
        infos[k].precision_used = p->cur;
        infos[k].refined = m[k].refined;
    }
    const double t = now_s() - t0;
    for (int k = 0; k < n; ++k) {
        infos[k].t_solve_s = t;
        infos[k].t_setup_s = b->probs[k]->t_setup;
    }
    return SPOCK_OK;
}

int32_t spock_batch_run_steps(spock_batch* b, int32_t prec, int32_t steps, int32_t sync) {
    if (!b || steps < 0 || (steps & 1)) return fail(SPOCK_E_INVALID, "steps must be even and >= 0");
    if (prec != SPOCK_FP64 && prec != SPOCK_FP32) return fail(SPOCK_E_INVALID, "precision");
    for (int k = 0; k < b->n; ++k) {
        spock_problem* p = b->probs[k];
        int32_t r = move_iterate(p, prec);
        if (!r) r = normalize_parity(p);
        if (!r) r = hipStreamSynchronize(p->stream) == hipSuccess ? SPOCK_OK : fail(SPOCK_E_HIP, "sync");
        if (r) return r;
    }
    int32_t r = upload_active(b, nullptr);
    if (!r) r = prec == SPOCK_FP64 ? batch_steps<double>(b, steps, false) : batch_steps<float>(b, steps, false);
    if (r) return r;
    if (sync) HIP_TRY(hipStreamSynchronize(b->stream));
    return SPOCK_OK;
}

int32_t spock_batch_time_kernels(spock_batch* b, int32_t prec, int32_t steps, double* ms_total, double* ms_k) {
    if (!b || steps < 2 || (steps & 1) || !ms_k) return fail(SPOCK_E_INVALID, "steps must be even and >= 2");
    int32_t r = spock_batch_run_steps(b, prec, 0, 1);
    if (r) return r;
    std::vector<hipEvent_t> ev(4 * (size_t)steps + 1);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventRecord(ev[0], b->stream));
    for (int k = 0; k < steps; ++k)
        for (int ph = 0; ph < 4; ++ph) {
            if (prec == SPOCK_FP64) HIP_TRY(spk::launch_phase<double>(b->d64, b->cfg64, ph, k & 1, 0, b->stream));
            else HIP_TRY(spk::launch_phase<float>(b->d32, b->cfg32, ph, k & 1, 0, b->stream));
            HIP_TRY(hipEventRecord(ev[4 * k + ph + 1], b->stream));
        }
    HIP_TRY(hipEventSynchronize(ev.back()));
    double t[4] = {0, 0, 0, 0};
    for (int k = 0; k < steps; ++k)
        for (int ph = 0; ph < 4; ++ph) {
            float a = 0;
            HIP_TRY(hipEventElapsedTime(&a, ev[4 * k + ph], ev[4 * k + ph + 1]));
            t[ph] += a;
        }
    float tot = 0;
    HIP_TRY(hipEventElapsedTime(&tot, ev[0], ev.back()));
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (ms_total) *ms_total = tot / steps;
    for (int ph = 0; ph < 4; ++ph) ms_k[ph] = t[ph] / steps;
    return read_all(b);
}

int32_t spock_batch_time_steps(spock_batch* b, int32_t prec, int32_t steps, double* ms_total, double* ms_b,
                               double* ms_f) {
    double k[4];
    int32_t r = spock_batch_time_kernels(b, prec, steps, ms_total, k);
    if (r) return r;
    if (ms_b) *ms_b = k[0] + k[1];
    if (ms_f) *ms_f = k[2] + k[3];
    return SPOCK_OK;
}

int32_t spock_batch_set_launch(spock_batch* b, int32_t precision, int32_t workgroup) {
    if (!b || !(workgroup == 64 || workgroup == 128 || workgroup == 256 || workgroup == 512))
        return fail(SPOCK_E_INVALID, "workgroup must be 64, 128, 256 or 512");
    const spk::LaunchCfg c = precision == SPOCK_FP64 ? batch_cfg<double>(b, workgroup) : batch_cfg<float>(b, workgroup);
    if (c.node_wg != workgroup) return fail(SPOCK_E_INVALID, "LDS too large");
    HIP_TRY(hipStreamSynchronize(b->stream));
    const int gi = precision == SPOCK_FP64 ? 0 : 1;
    if (b->graph[gi]) {
        (void)hipGraphExecDestroy(b->graph[gi]);
        b->graph[gi] = nullptr;
        b->graph_steps[gi] = 0;
    }
    if (precision == SPOCK_FP64) b->cfg64 = c;
    else b->cfg32 = c;
    return SPOCK_OK;
}

int32_t spock_batch_step_bytes(const spock_batch* b, int32_t prec, double* bb, double* bf) {
    if (!b) return fail(SPOCK_E_INVALID, "null batch");
    const int q = prec == SPOCK_FP64 ? 0 : 1;
    if (bb) *bb = b->bytes_k[q][0] + b->bytes_k[q][1];
    if (bf) *bf = b->bytes_k[q][2] + b->bytes_k[q][3];
    return SPOCK_OK;
}

int32_t spock_batch_kernel_bytes(const spock_batch* b, int32_t prec, double* bytes) {
    if (!b || !bytes) return fail(SPOCK_E_INVALID, "null argument");
    const int q = prec == SPOCK_FP64 ? 0 : 1;
    for (int ph = 0; ph < 4; ++ph) bytes[ph] = b->bytes_k[q][ph];
    return SPOCK_OK;
}

}  // extern "C"
