// Serving loop: continuous batching of annealing requests on one GPU.
//
// Requests queue in arrival order.  A request is admitted when a slot is
// free and its estimated device footprint (couplings plus replica state)
// fits the memory budget next to the requests already running; its replica
// state then stays resident until it retires.  The service thread runs
// scheduling rounds: each round advances every running request by one chunk
// of steps -- the column-split instances packed into one cooperative launch
// that has the device to itself (its workgroups wait for each other), then
// all running instances with N <= 512 in one batched launch on the service
// stream, overlapped with the VALU sweeps (ELL, FP32, few replicas), whose
// own launches go round-robin to three more streams -- then reads every
// request's best energy with one synchronisation.  A request retires when its best energy reaches its
// target or its step budget is used up; its result (energy, replica, steps,
// best state, timestamps) is kept for the caller and its device state is
// released, which may admit waiting requests at the next round.  Requests
// stop only at chunk boundaries, so a request's result is the same alone and
// in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

#include "phia.h"
#include "phia_internal.h"
#include "phia_problem.h"

using namespace phia;

namespace {

struct Request {
    uint64_t ticket = 0;
    phia_problem* p = nullptr;
    int32_t R = 0;
    int64_t max_steps = 0;
    int64_t target = 0;
    phia_schedule sched{};
    std::vector<float> betas;  // copy of an explicit table
    uint64_t seed = 0;
    size_t footprint = 0;
    hipStream_t saved_stream = nullptr;
    phia_result res{};
    std::vector<int8_t> spins;
    std::atomic<bool> cancel{false};
    bool started = false;   // service thread only
    bool failed = false;    // service thread only
    int64_t energy = INT64_MAX;  // service thread only: best energy of the last round
    int32_t replica = -1;        // service thread only
};

}  // namespace

struct phia_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> running;
    std::unordered_map<uint64_t, Request*> all;
    size_t budget = 0, in_use = 0;
    int max_slots = 1;
    int64_t chunk = 1000;
    int dev = 0;
    hipStream_t st = nullptr;
    static constexpr int kAux = 3;  // streams for the VALU sweeps' own launches (default priority)
    hipStream_t aux[kAux] = {};
    hipEvent_t ev_split = nullptr;      // the cooperative launch of a round has ended
    hipEvent_t ev_aux[kAux] = {};       // an auxiliary stream's launches of a round have ended
    int64_t* host_res = nullptr;  // pinned: [2 n] (energy, replica) of a round's n requests, then [n] int32 error words
    int64_t* dev_res = nullptr;   // the same on the device, written by one batched argmin per round
    SweepArgs* dtab = nullptr;  // work table of the batched small instances
    size_t dtab_cap = 0;
    SweepArgs* gtab = nullptr;  // work table of the column-split instances
    size_t gtab_cap = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

size_t footprint(const phia_problem* p, int32_t R, int64_t T, bool mh = false)
{
    const size_t RN = static_cast<size_t>(R) * p->Np;
    // the couplings count whether or not they are resident yet
    size_t b = p->jres_bytes + RN * 9 + static_cast<size_t>(R) * 16 + static_cast<size_t>(T) * 4 +
               2 * RN / 16 * 8 * 2 + 65536;
    // accept/reject: x snapshot, per-replica state, beta table, kinetic units per member
    if (mh) b += RN * 4 + static_cast<size_t>(R) * 32 + static_cast<size_t>(T) * 4 + RN / 16 * 8 * 2;
    return b;
}

void finish(phia_server* s, Request* r, int32_t state)
{
    r->res.state = state;
    r->res.t_done = s->now();
    r->res.steps_used = r->p->k;
    if (r->started) free_state(r->p);
    if (r->p->defer) release_resident(r->p);
    r->p->st = r->saved_stream;
    r->p->one_block_kernel = false;
    r->p->started = false;
    r->p->has_run = false;
    s->in_use -= r->footprint;
}

// One scheduling round over the running requests (service thread only).
void round_once(phia_server* s, std::vector<Request*>& run)
{
    const int n = static_cast<int>(run.size());
    std::vector<phia_problem*> small, split;
    std::vector<int64_t> small_end, split_end;
    std::vector<std::pair<Request*, int64_t>> solo;  // VALU sweeps (normal launches of their own)
    hipError_t e = hipSuccess;
    for (Request* r : run) {
        phia_problem* p = r->p;
        const int64_t k_end = std::min(p->k + s->chunk, p->T);
        const bool mfma = p->path == PHIA_PATH_I8 || p->path == PHIA_PATH_BF16HILO;
        if (p->Np <= kBatchMaxNp && mfma) {
            small.push_back(p);
            small_end.push_back(k_end);
        } else if (mfma && p->geo.kind == 0 && p->geo.G > 1) {
            split.push_back(p);
            split_end.push_back(k_end);
        } else if (k_end > p->k) {
            if (p->geo.kind == 4)
                solo.push_back({r, k_end});
            else if (phia_anneal_run(p, k_end) != PHIA_OK)
                r->failed = true;
        }
    }
    // Column-split instances: several per cooperative launch, with nothing
    // else on the device (the launches below wait for it).
    if (!split.empty() && launch_group_chunk(split.data(), static_cast<int>(split.size()), split_end.data(), s->st,
                                             s->gtab, s->gtab_cap) != PHIA_OK)
        for (Request* r : run)
            if (std::find(split.begin(), split.end(), r->p) != split.end()) r->failed = true;
    // The VALU sweeps' launches on the auxiliary streams, after it.
    const int na = std::min<int>(phia_server::kAux, static_cast<int>(solo.size()));
    bool aux_ok = na == 0 || hipEventRecord(s->ev_split, s->st) == hipSuccess;
    for (int k = 0; aux_ok && k < na; ++k) aux_ok = hipStreamWaitEvent(s->aux[k], s->ev_split, 0) == hipSuccess;
    for (size_t i = 0; i < solo.size(); ++i) {
        Request* r = solo[i].first;
        if (!aux_ok) {
            r->failed = true;
            continue;
        }
        r->p->st = s->aux[i % na];
        if (phia_anneal_run(r->p, solo[i].second) != PHIA_OK) r->failed = true;
        r->p->st = s->st;
    }
    // The batched small instances on the service stream, beside them.
    if (!small.empty() && launch_batch_chunk(small.data(), static_cast<int>(small.size()), small_end.data(), s->st,
                                             s->dtab, s->dtab_cap) != PHIA_OK)
        for (Request* r : run)
            if (std::find(small.begin(), small.end(), r->p) != small.end()) r->failed = true;
    // The service stream waits for the auxiliary ones before the argmins.
    for (int k = 0; k < na; ++k)
        if (hipEventRecord(s->ev_aux[k], s->aux[k]) != hipSuccess ||
            hipStreamWaitEvent(s->st, s->ev_aux[k], 0) != hipSuccess) {
            for (auto& q : solo) q.first->failed = true;
            break;
        }
    // Every request's best (energy, replica) and error word: one launch, one copy.
    std::vector<const int64_t*> best(n);
    std::vector<const int32_t*> errw(n);
    std::vector<int32_t> reps(n);
    for (int i = 0; i < n; ++i) {
        const phia_problem* p = run[i]->p;
        best[i] = p->dbestE;
        reps[i] = p->R;
        errw[i] = p->geo.G > 1 ? p->derr : nullptr;
    }
    int32_t* dev_err = reinterpret_cast<int32_t*>(s->dev_res + 2 * n);
    const size_t res_bytes = sizeof(int64_t) * 2 * n + sizeof(int32_t) * n;
    if (n > 0 && ((e = launch_argmin_many(best.data(), reps.data(), errw.data(), n, s->dev_res, dev_err, s->st)) !=
                      hipSuccess ||
                  (e = hipMemcpyAsync(s->host_res, s->dev_res, res_bytes, hipMemcpyDeviceToHost, s->st)) !=
                      hipSuccess))
        for (Request* r : run) r->failed = true;
    e = hipStreamSynchronize(s->st);
    for (int k = 0; k < na; ++k) {  // complete already, unless an event call above failed
        const hipError_t ek = hipStreamSynchronize(s->aux[k]);
        if (e == hipSuccess) e = ek;
    }
    if (e != hipSuccess) {
        for (Request* r : run) {
            r->failed = true;
            r->p->poisoned = true;
        }
        return;
    }
    const int32_t* host_err = reinterpret_cast<const int32_t*>(s->host_res + 2 * n);
    for (int i = 0; i < n; ++i) {
        Request* r = run[i];
        if (r->failed) continue;
        if (host_err[i] != 0) {
            r->failed = true;
            r->p->poisoned = true;
            continue;
        }
        r->energy = s->host_res[2 * i];
        r->replica = static_cast<int32_t>(s->host_res[2 * i + 1]);
    }
}

void release_streams(phia_server* s)
{
    if (s->st) (void)hipStreamDestroy(s->st);
    for (int k = 0; k < phia_server::kAux; ++k) {
        if (s->aux[k]) (void)hipStreamDestroy(s->aux[k]);
        if (s->ev_aux[k]) (void)hipEventDestroy(s->ev_aux[k]);
    }
    if (s->ev_split) (void)hipEventDestroy(s->ev_split);
}

void service(phia_server* s)
{
    (void)hipSetDevice(s->dev);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // Admission in arrival order, within the slot count and the budget.
        std::vector<Request*> admitted;
        while (!s->pending.empty() && static_cast<int>(s->running.size()) < s->max_slots) {
            Request* r = s->pending.front();
            if (r->cancel) {
                s->pending.pop_front();
                r->res.state = PHIA_REQ_CANCELLED;
                r->res.t_done = s->now();
                continue;
            }
            if (s->in_use + r->footprint > s->budget) {
                if (s->running.empty()) {  // can never fit
                    s->pending.pop_front();
                    r->res.state = PHIA_REQ_FAILED;
                    r->res.t_done = s->now();
                    continue;
                }
                break;
            }
            s->pending.pop_front();
            s->in_use += r->footprint;
            r->res.state = PHIA_REQ_RUNNING;
            r->res.t_admit = s->now();
            s->running.push_back(r);
            admitted.push_back(r);
        }
        s->cv_done.notify_all();
        if (s->running.empty()) {
            if (s->stop) break;
            s->cv_work.wait(lk);
            continue;
        }
        std::vector<Request*> run = s->running;
        lk.unlock();
        for (Request* r : admitted) {
            r->saved_stream = r->p->st;
            r->p->st = s->st;
            r->p->one_block_kernel = true;  // geometries that the table launches carry
            if (phia_anneal_start(r->p, r->R, r->max_steps, &r->sched, r->seed) != PHIA_OK)
                r->failed = true;
            else
                r->started = true;
        }
        std::vector<Request*> live;
        for (Request* r : run)
            if (!r->failed) live.push_back(r);
        round_once(s, live);
        // Retire finished requests (their best state is copied out first).
        std::vector<std::tuple<Request*, int32_t, bool>> done;
        for (Request* r : run) {
            if (r->failed) {
                done.push_back({r, PHIA_REQ_FAILED, false});
                continue;
            }
            const bool hit = r->energy <= r->target;
            const bool cancel = r->cancel.load();
            if (hit || r->p->k >= r->p->T || cancel) {
                if (r->p->has_run && r->replica >= 0) {
                    r->spins.resize(static_cast<size_t>(r->p->N));
                    (void)hipMemcpy(r->spins.data(), r->p->dbestS + static_cast<size_t>(r->replica) * r->p->Np,
                                    static_cast<size_t>(r->p->N), hipMemcpyDeviceToHost);
                }
                done.push_back({r, cancel && !hit ? PHIA_REQ_CANCELLED : PHIA_REQ_DONE, hit});
            }
        }
        lk.lock();
        for (Request* r : run) {
            r->res.energy_units = r->energy;
            r->res.replica = r->replica;
            r->res.steps_used = r->p->k;
        }
        for (auto& d : done) {
            Request* r = std::get<0>(d);
            r->res.success = std::get<2>(d) ? 1 : 0;
            finish(s, r, std::get<1>(d));
            s->running.erase(std::find(s->running.begin(), s->running.end(), r));
        }
        if (!done.empty()) s->cv_done.notify_all();
    }
    s->cv_done.notify_all();
}

}  // namespace

extern "C" {

phia_status phia_server_create(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, int32_t device,
                               phia_server** out)
{
    clear_error();
    if (!out) return fail(PHIA_EINVAL, "out is null");
    *out = nullptr;
    if (hbm_budget == 0 || max_slots < 1 || max_slots > 65536 || chunk_steps < 1)
        return fail(PHIA_EINVAL, "bad server parameters");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(PHIA_EINVAL, "device %d not present", device);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    phia_server* s = new (std::nothrow) phia_server();
    if (!s) return fail(PHIA_ENOMEM, "host allocation failed");
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->chunk = chunk_steps;
    s->dev = device;
    s->t0 = std::chrono::steady_clock::now();
    e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    for (int k = 0; e == hipSuccess && k < phia_server::kAux; ++k) {
        e = hipStreamCreateWithFlags(&s->aux[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_aux[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_split, hipEventDisableTiming);
    const size_t res_bytes = sizeof(int64_t) * 2 * max_slots + sizeof(int32_t) * max_slots;
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->host_res), res_bytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->dev_res), res_bytes);
    if (e != hipSuccess) {
        if (s->host_res) (void)hipHostFree(s->host_res);
        release_streams(s);
        delete s;
        return hip_fail(nullptr, e, "server resources");
    }
    s->worker = std::thread(service, s);
    *out = s;
    return PHIA_OK;
}

phia_status phia_server_submit(phia_server* s, phia_problem* p, int32_t replicas, int64_t max_steps,
                               int64_t target_energy_units, const phia_schedule* sched, uint64_t seed,
                               uint64_t* ticket)
{
    clear_error();
    if (!s || !ticket) return fail(PHIA_EINVAL, "null argument");
    phia_status st = check_owned(p);
    if (st != PHIA_OK) return st;
    if ((st = check_schedule(replicas, max_steps, sched)) != PHIA_OK) return st;
    if (sched->initial_kick) return fail(PHIA_EINVAL, "served requests run without the initial kick");
    if (p->dev != s->dev) return fail(PHIA_EINVAL, "problem is on another device");
    Request* r = new (std::nothrow) Request();
    if (!r) return fail(PHIA_ENOMEM, "host allocation failed");
    r->p = p;
    r->R = replicas;
    r->max_steps = max_steps;
    r->target = target_energy_units;
    r->sched = *sched;
    if (sched->betas) {
        r->betas.assign(sched->betas, sched->betas + max_steps);
        r->sched.betas = r->betas.data();
    }
    r->seed = seed;
    r->footprint = footprint(p, replicas, max_steps, sched->metropolis != 0);
    r->res.state = PHIA_REQ_QUEUED;
    r->res.energy_units = INT64_MAX;
    r->res.frac_bits = p->f;
    r->res.replica = -1;
    r->res.t_admit = -1.0;
    r->res.t_done = -1.0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& kv : s->all)
            if (kv.second->p == p && (kv.second->res.state == PHIA_REQ_QUEUED ||
                                      kv.second->res.state == PHIA_REQ_RUNNING)) {
                delete r;
                return fail(PHIA_EINVAL, "problem already has an unfinished request");
            }
        r->ticket = s->next_ticket++;
        r->res.t_arrive = s->now();
        s->all[r->ticket] = r;
        s->pending.push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return PHIA_OK;
}

phia_status phia_server_footprint(const phia_problem* p, int32_t replicas, int64_t max_steps, size_t* bytes)
{
    clear_error();
    if (!p || !bytes || replicas < 1 || max_steps < 1) return fail(PHIA_EINVAL, "bad argument");
    *bytes = footprint(p, replicas, max_steps);
    return PHIA_OK;
}

phia_status phia_server_poll(phia_server* s, uint64_t ticket, phia_result* out)
{
    clear_error();
    if (!s || !out) return fail(PHIA_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(PHIA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    *out = it->second->res;
    return PHIA_OK;
}

phia_status phia_server_wait(phia_server* s, uint64_t ticket, double timeout_s, phia_result* out)
{
    clear_error();
    if (!s || !out) return fail(PHIA_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(PHIA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second;
    auto finished = [&] { return r->res.state != PHIA_REQ_QUEUED && r->res.state != PHIA_REQ_RUNNING; };
    if (timeout_s < 0)
        s->cv_done.wait(lk, finished);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
        *out = r->res;
        return fail(PHIA_ESTATE, "request %llu not finished within the timeout", (unsigned long long)ticket);
    }
    *out = r->res;
    return PHIA_OK;
}

phia_status phia_server_spins(phia_server* s, uint64_t ticket, int8_t* spins)
{
    clear_error();
    if (!s || !spins) return fail(PHIA_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(PHIA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Request* r = it->second;
    if (r->res.state != PHIA_REQ_DONE && r->res.state != PHIA_REQ_CANCELLED) return fail(PHIA_ESTATE, "not done");
    if (r->spins.empty()) return fail(PHIA_ESTATE, "no steps ran");
    std::memcpy(spins, r->spins.data(), r->spins.size());
    return PHIA_OK;
}

phia_status phia_server_cancel(phia_server* s, uint64_t ticket)
{
    clear_error();
    if (!s) return fail(PHIA_EINVAL, "null argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return fail(PHIA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        it->second->cancel = true;
    }
    s->cv_work.notify_one();
    return PHIA_OK;
}

void phia_server_destroy(phia_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Request* r : s->pending) r->cancel = true;
        for (Request* r : s->running) r->cancel = true;
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->dev);
    for (auto& kv : s->all) delete kv.second;
    if (s->dtab) (void)hipFree(s->dtab);
    if (s->gtab) (void)hipFree(s->gtab);
    if (s->host_res) (void)hipHostFree(s->host_res);
    if (s->dev_res) (void)hipFree(s->dev_res);
    release_streams(s);
    delete s;
}

}  // extern "C"
