// Continuous-batching solve server.
//
// Requests (mesh + charges + options) are queued in arrival order.  A request
// is admitted as soon as a slot is free and its estimated device footprint
// fits in what the budget leaves beside the requests already running (first
// fit in arrival order).  Every admitted request runs on its own worker
// thread with its own mesh handle, HIP stream and stream-ordered allocations,
// so requests of different sizes overlap on the device while each one's
// arithmetic is exactly what it would be alone (no shared buffers, fixed
// reduction orders): a result does not depend on its co-tenants.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "pbm_internal.h"

namespace pbm {
DevMesh *create_mesh_checked(const pb_mesh *mesh, const pb_options *opt, BlockCache *cache);
size_t estimate_device_bytes(int V, int T, const pb_options *opt);
}  // namespace pbm

using namespace pbm;

namespace {

struct Request {
    uint64_t id = 0;
    std::vector<double> xyz, qxyz, q;
    std::vector<int32_t> tri;
    pb_options opt{};
    size_t est = 0;
    int state = 0;   // 0 queued, 1 running, 2 done, 3 cancelled
    pb_status status = PB_OK;
    std::string err;
    pb_result res{};
    std::vector<double> phi, dphi;
    double t_submit = 0, t_start = 0, t_end = 0;
};

double clock_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct pb_server {
    size_t budget = 0;
    int slots = 1;
    double t0 = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    size_t inflight = 0, peak_inflight = 0;
    int running = 0, peak_running = 0;
    int64_t submitted = 0, completed = 0, cancelled = 0, failed = 0;
    uint64_t next_id = 1;
    bool stop = false;
    BlockCache *cache = nullptr;   // large device blocks kept between requests (null without a device)
    std::vector<std::thread> workers;

    Request *pick()
    {
        for (auto it = queue.begin(); it != queue.end(); ++it)
            if (inflight + (*it)->est <= budget) {
                Request *r = *it;
                queue.erase(it);
                return r;
            }
        return nullptr;
    }

    void run(Request *r)
    {
        pb_mesh m{(int32_t)(r->xyz.size() / 3), (int32_t)(r->tri.size() / 3), r->xyz.data(), r->tri.data()};
        pb_charges c{(int32_t)r->q.size(), r->qxyz.data(), r->q.data()};
        r->phi.assign(m.n_vertices, 0.0);
        r->dphi.assign(m.n_vertices, 0.0);
        r->res.phi = r->phi.data();
        r->res.dphi = r->dphi.data();
        try {
            std::unique_ptr<DevMesh> d(create_mesh_checked(&m, &r->opt, cache));
            r->status = solve_on_mesh(*d, &c, &r->res);
        } catch (const Error &e) {
            r->status = e.code;
            r->err = e.msg;
        } catch (...) {
            r->status = PB_E_DEVICE;
            r->err = "unexpected internal error";
        }
    }

    void worker()
    {
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop) return true;
                    r = pick();
                    return r != nullptr;
                });
                if (!r) return;   // stopping
                r->state = 1;
                r->t_start = clock_s() - t0;
                inflight += r->est;
                ++running;
                peak_inflight = std::max(peak_inflight, inflight);
                peak_running = std::max(peak_running, running);
            }
            run(r);
            {
                std::lock_guard<std::mutex> lk(mu);
                r->t_end = clock_s() - t0;
                inflight -= r->est;
                --running;
                r->state = 2;
                ++completed;
                if (r->status < 0) ++failed;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

#define SV_TRY try {
#define SV_CATCH                              \
    }                                         \
    catch (const Error &e) {                  \
        set_error(e.msg);                     \
        return e.code;                        \
    }                                         \
    catch (const std::bad_alloc &) {          \
        set_error("host out of memory");      \
        return PB_E_NOMEM;                    \
    }                                         \
    catch (...) {                             \
        set_error("unexpected internal error"); \
        return PB_E_DEVICE;                   \
    }

extern "C" {

pb_status pb_estimate_device_bytes(const pb_mesh *mesh, const pb_options *opt, size_t *bytes)
{
    SV_TRY
    if (!mesh || !opt || !bytes) fail(PB_E_INVALID_ARG, "NULL argument");
    *bytes = estimate_device_bytes(mesh->n_vertices, mesh->n_triangles, opt);
    return PB_OK;
    SV_CATCH
}

pb_status pb_server_create(size_t hbm_budget, int32_t max_slots, pb_server **out)
{
    SV_TRY
    if (!out || max_slots < 1 || max_slots > 64) fail(PB_E_INVALID_ARG, "max_slots must be in [1, 64]");
    *out = nullptr;
    size_t budget = hbm_budget;
    if (budget == 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(PB_E_DEVICE, "no HIP device available");
        HIPCHECK(hipSetDevice(0));
        size_t freeb = 0, total = 0;
        HIPCHECK(hipMemGetInfo(&freeb, &total));
        budget = (size_t)(0.9 * (double)freeb);
    }
    std::unique_ptr<pb_server> s(new pb_server());
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) s->cache = block_cache_create(budget);
    s->budget = budget;
    s->slots = max_slots;
    s->t0 = clock_s();
    pb_server *sp = s.get();
    for (int k = 0; k < max_slots; ++k) s->workers.emplace_back([sp] { sp->worker(); });
    *out = s.release();
    return PB_OK;
    SV_CATCH
}

pb_status pb_server_destroy(pb_server *s)
{
    SV_TRY
    if (!s) return PB_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Request *r : s->queue) {
            r->state = 3;
            ++s->cancelled;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    block_cache_destroy(s->cache);
    delete s;
    return PB_OK;
    SV_CATCH
}

pb_status pb_submit(pb_server *s, const pb_mesh *mesh, const pb_charges *charges, const pb_options *opt,
                    uint64_t *ticket)
{
    SV_TRY
    if (!s || !mesh || !charges || !opt || !ticket) fail(PB_E_INVALID_ARG, "NULL argument");
    if (!mesh->xyz || !mesh->tri || mesh->n_vertices < 4 || mesh->n_triangles < 4)
        fail(PB_E_INVALID_ARG, "bad mesh");
    if (!charges->xyz || !charges->q || charges->n < 1) fail(PB_E_INVALID_ARG, "bad charges");
    std::unique_ptr<Request> r(new Request());
    r->xyz.assign(mesh->xyz, mesh->xyz + 3 * (size_t)mesh->n_vertices);
    r->tri.assign(mesh->tri, mesh->tri + 3 * (size_t)mesh->n_triangles);
    r->qxyz.assign(charges->xyz, charges->xyz + 3 * (size_t)charges->n);
    r->q.assign(charges->q, charges->q + charges->n);
    r->opt = *opt;
    r->est = estimate_device_bytes(mesh->n_vertices, mesh->n_triangles, opt);
    if (r->est > s->budget) fail(PB_E_NOMEM, "request footprint exceeds the server's device-memory budget");
    // the handle may not outgrow its admission footprint
    if (r->opt.memory_budget == 0 || r->opt.memory_budget > r->est) r->opt.memory_budget = r->est;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) fail(PB_E_STATE, "server is shutting down");
    r->id = s->next_id++;
    r->t_submit = clock_s() - s->t0;
    *ticket = r->id;
    s->queue.push_back(r.get());
    s->all.emplace(r->id, std::move(r));
    ++s->submitted;
    s->cv_work.notify_one();
    return PB_OK;
    SV_CATCH
}

pb_status pb_poll(pb_server *s, uint64_t ticket, int32_t *done)
{
    SV_TRY
    if (!s || !done) fail(PB_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) fail(PB_E_INVALID_ARG, "unknown ticket");
    *done = it->second->state >= 2 ? 1 : 0;
    return PB_OK;
    SV_CATCH
}

pb_status pb_cancel(pb_server *s, uint64_t ticket)
{
    SV_TRY
    if (!s) fail(PB_E_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) fail(PB_E_INVALID_ARG, "unknown ticket");
    Request *r = it->second.get();
    if (r->state != 0) fail(PB_E_STATE, "request is already running or finished");
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
        if (*q == r) {
            s->queue.erase(q);
            break;
        }
    r->state = 3;
    ++s->cancelled;
    s->cv_done.notify_all();
    return PB_OK;
    SV_CATCH
}

pb_status pb_wait(pb_server *s, uint64_t ticket, pb_result *out, pb_request_times *times)
{
    SV_TRY
    if (!s || !out) fail(PB_E_INVALID_ARG, "NULL argument");
    std::unique_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) fail(PB_E_INVALID_ARG, "unknown ticket");
        Request *rp = it->second.get();
        s->cv_done.wait(lk, [&] { return rp->state >= 2; });
        r = std::move(it->second);
        s->all.erase(it);
    }
    if (times) {
        times->t_submit = r->t_submit;
        times->t_start = r->t_start;
        times->t_end = r->t_end;
    }
    if (r->state == 3) fail(PB_E_STATE, "request was cancelled");
    if (r->status < 0) fail(r->status, r->err);
    double *phi = out->phi, *dphi = out->dphi;
    *out = r->res;
    out->phi = phi;
    out->dphi = dphi;
    if (phi) std::copy(r->phi.begin(), r->phi.end(), phi);
    if (dphi) std::copy(r->dphi.begin(), r->dphi.end(), dphi);
    return r->status;
    SV_CATCH
}

pb_status pb_server_get_stats(pb_server *s, pb_server_stats *st)
{
    SV_TRY
    if (!s || !st) fail(PB_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->cancelled = s->cancelled;
    st->failed = s->failed;
    st->running = s->running;
    st->queued = (int32_t)s->queue.size();
    st->peak_running = s->peak_running;
    st->inflight_bytes = s->inflight;
    st->peak_inflight_bytes = s->peak_inflight;
    st->budget = s->budget;
    return PB_OK;
    SV_CATCH
}

}  // extern "C"
