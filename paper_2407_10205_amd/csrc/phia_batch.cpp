// Batched sweep: many instances of uneven size annealed by one captured
// HIP graph.  Every instance is split into 16-replica work items; one
// workgroup runs one item for all of its steps with all of its columns (no
// exchange between workgroups), its coupling slice in LDS when it fits and
// streamed from L2 otherwise.  Items are grouped into buckets by (path,
// column blocks per wave, J placement), each bucket sorted largest first so
// that the dispatcher balances the tail; the init kernel and the bucket
// kernels are captured into one graph and launched once.  Results are
// bit-identical to annealing each instance alone: the Gaussian stream is
// keyed by (seed, replica) and the sweep's arithmetic does not depend on the
// launch geometry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "phia.h"
#include "phia_internal.h"
#include "phia_problem.h"

using namespace phia;

namespace {

struct Bucket {
    int path = 0, cbw = 2, jl = 1, mh = 0;
    size_t lds = 0;
    std::vector<SweepArgs> items;
};

// Work items of steps [p->k, k_end) of problem p, added to its bucket.
void add_items(phia_problem* p, int64_t k_end, std::map<std::tuple<int, int, int, int>, Bucket>& buckets)
{
    const int ncb = p->Np / 16;
    const int cbw = ncb <= kWaves * 2 ? 2 : 4;
    const int jl = sweep_batch_lds_bytes(p->path, p->Np, 1, p->mh) <= static_cast<size_t>(kLdsMax) ? 1 : 0;
    const int nblocks = (p->R + 15) / 16;
    SweepArgs a = sweep_args(p);
    a.inc = 0;  // table launches carry no flip-incremental variant
    a.J = p->dJ;  // int8 fragments (the batch kernel's operands)
    a.k0 = p->k;
    a.k1 = k_end;
    a.etrace = nullptr;
    a.G = 1;
    a.ncb = ncb;
    a.rows = 16;
    a.j_lds = jl;
    Bucket& b = buckets[std::make_tuple(p->path, cbw, jl, p->mh)];
    b.path = p->path;
    b.cbw = cbw;
    b.jl = jl;
    b.mh = p->mh;
    b.lds = std::max(b.lds, sweep_batch_lds_bytes(p->path, p->Np, jl, p->mh));
    for (int blk = 0; blk < nblocks; ++blk) {
        SweepArgs it = a;
        it.block = blk;
        it.nblocks = blk + 1;
        it.ngroups = 1;
        b.items.push_back(it);
    }
}

// Largest instances first (the dispatcher then fills the tail with small
// ones), and within every run of 8 instances with the same item count the
// items interleaved so that the items of one instance sit 8 workgroups apart:
// under round-robin dispatch over the 8 XCDs they share one XCD and its L2,
// which then streams that instance's J once for all of its items.
void order_items(std::vector<SweepArgs>& items)
{
    std::stable_sort(items.begin(), items.end(), [](const SweepArgs& x, const SweepArgs& y) { return x.Np > y.Np; });
    std::vector<std::pair<size_t, size_t>> inst;  // (first item, item count), items of one instance are adjacent
    for (size_t i = 0; i < items.size();) {
        size_t j = i + 1;
        while (j < items.size() && items[j].x == items[i].x) ++j;
        inst.emplace_back(i, j - i);
        i = j;
    }
    std::vector<SweepArgs> out;
    out.reserve(items.size());
    for (size_t c = 0; c < inst.size(); c += 8) {
        const size_t n = std::min<size_t>(8, inst.size() - c);
        bool same = n == 8;
        for (size_t k = 1; same && k < n; ++k) same = inst[c + k].second == inst[c].second;
        if (same) {
            for (size_t b = 0; b < inst[c].second; ++b)
                for (size_t k = 0; k < n; ++k) out.push_back(items[inst[c + k].first + b]);
        } else {
            for (size_t k = 0; k < n; ++k)
                for (size_t b = 0; b < inst[c + k].second; ++b) out.push_back(items[inst[c + k].first + b]);
        }
    }
    items.swap(out);
}

}  // namespace

namespace phia {

// Enqueue steps [k, k_end[i]) of every problem as batch work items on st
// (problems already started, Np <= kBatchMaxNp, matrix-core paths).  The
// device table `dtab` (capacity `cap` entries, grown as needed) must not be
// in use by earlier launches; the caller synchronises between rounds.
phia_status launch_batch_chunk(phia_problem* const* probs, int count, const int64_t* k_end, hipStream_t st,
                               SweepArgs*& dtab, size_t& cap)
{
    std::map<std::tuple<int, int, int, int>, Bucket> buckets;
    for (int i = 0; i < count; ++i)
        if (k_end[i] > probs[i]->k) add_items(probs[i], k_end[i], buckets);
    std::vector<SweepArgs> tab;
    std::vector<size_t> offs;
    for (auto& kv : buckets) {
        order_items(kv.second.items);
        offs.push_back(tab.size());
        tab.insert(tab.end(), kv.second.items.begin(), kv.second.items.end());
    }
    if (tab.empty()) return PHIA_OK;
    hipError_t e;
    if (tab.size() > cap) {
        if (dtab) (void)hipFree(dtab);
        dtab = nullptr;
        cap = 0;
        if ((e = hipMalloc(&dtab, sizeof(SweepArgs) * tab.size() * 2)) != hipSuccess)
            return fail(PHIA_ENOMEM, "work table allocation failed");
        cap = tab.size() * 2;
    }
    // pageable source: the copy completes before hipMemcpy returns
    if ((e = hipMemcpy(dtab, tab.data(), sizeof(SweepArgs) * tab.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(nullptr, e, "work table upload");
    size_t bi = 0;
    for (auto& kv : buckets) {
        if ((e = prepare_sweep_batch(kv.second.path, kv.second.cbw, kv.second.mh, kv.second.lds)) != hipSuccess ||
            (e = launch_sweep_batch(kv.second.path, kv.second.cbw, kv.second.mh, dtab + offs[bi],
                                    static_cast<int>(kv.second.items.size()), kv.second.lds, st)) != hipSuccess)
            return hip_fail(nullptr, e, "batch chunk launch");
        ++bi;
    }
    for (int i = 0; i < count; ++i)
        if (k_end[i] > probs[i]->k) {
            probs[i]->k = k_end[i];
            probs[i]->has_run = true;
        }
    return PHIA_OK;
}

// Steps [p->k, k_end[i]) of column-split problems (k_sweep_mfma geometry with
// G > 1), several problems per cooperative launch: one table entry per
// workgroup, all of a problem's workgroups in one launch, launches packed up
// to the co-resident workgroup count.  Problems that cannot share a launch
// run alone.
phia_status launch_group_chunk(phia_problem* const* probs, int count, const int64_t* k_end, hipStream_t st,
                               SweepArgs*& dtab, size_t& cap)
{
    struct Launch {
        int path, mt, cbw, mh;
        size_t lds;
        std::vector<int> members;  // problem indices
        int nwg;
    };
    std::map<std::tuple<int, int, int, int>, std::vector<int>> by_kernel;
    for (int i = 0; i < count; ++i) {
        const phia_problem* p = probs[i];
        if (k_end[i] <= p->k) continue;
        if (p->geo.kind != 0 || p->geo.G < 2) return fail(PHIA_EINVAL, "problem %d is not a column-split sweep", i);
        by_kernel[std::make_tuple(p->path, p->geo.mt, p->geo.cbw, p->mh)].push_back(i);
    }
    std::vector<Launch> launches;
    std::vector<int> alone;
    for (auto& kv : by_kernel) {
        size_t lds = 0;
        for (int i : kv.second) lds = std::max(lds, probs[i]->geo.lds);
        const int maxwg = max_coresident_group_table(std::get<0>(kv.first), std::get<1>(kv.first),
                                                     std::get<2>(kv.first), std::get<3>(kv.first), lds);
        Launch cur{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first), lds,
                   {}, 0};
        for (int i : kv.second) {
            const int w = probs[i]->geo.ngroups * probs[i]->geo.G;
            if (w > maxwg) {
                alone.push_back(i);
                continue;
            }
            if (cur.nwg + w > maxwg) {
                launches.push_back(cur);
                cur.members.clear();
                cur.nwg = 0;
            }
            cur.members.push_back(i);
            cur.nwg += w;
        }
        if (!cur.members.empty()) launches.push_back(cur);
    }
    std::vector<SweepArgs> tab;
    std::vector<size_t> offs;
    hipError_t e;
    for (const Launch& L : launches) {
        offs.push_back(tab.size());
        for (int i : L.members) {
            phia_problem* p = probs[i];
            // 32-bit tags: restart the sequence (cleared words) before it would wrap
            const uint64_t iters = static_cast<uint64_t>((p->geo.nblocks + p->geo.ngroups - 1) / p->geo.ngroups);
            if (static_cast<uint64_t>(p->seq) + iters * static_cast<uint64_t>(k_end[i] - p->k + 1) > 0xfffffffeull) {
                if ((e = clear_exchange(p)) != hipSuccess) return hip_fail(p, e, "exchange reset");
                p->seq = 0;
            }
            SweepArgs a = sweep_args(p);
            a.inc = 0;  // table launches carry no flip-incremental variant
            a.k0 = p->k;
            a.k1 = k_end[i];
            a.etrace = nullptr;
            a.xcd_map = 0;
            for (int g = 0; g < p->geo.ngroups; ++g)
                for (int m = 0; m < p->geo.G; ++m) {
                    SweepArgs it = a;
                    it.block = g;
                    it.member = m;
                    tab.push_back(it);
                }
        }
    }
    if (!tab.empty()) {
        if (tab.size() > cap) {
            if (dtab) (void)hipFree(dtab);
            dtab = nullptr;
            cap = 0;
            if ((e = hipMalloc(&dtab, sizeof(SweepArgs) * tab.size() * 2)) != hipSuccess)
                return fail(PHIA_ENOMEM, "work table allocation failed");
            cap = tab.size() * 2;
        }
        if ((e = hipMemcpy(dtab, tab.data(), sizeof(SweepArgs) * tab.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(nullptr, e, "work table upload");
    }
    for (size_t li = 0; li < launches.size(); ++li) {
        const Launch& L = launches[li];
        // test hook, as in phia_anneal_run: the error word raised before the
        // launch, as if another workgroup had given up
        for (int i : L.members)
            if (probs[i]->give_up && (e = hipMemsetAsync(probs[i]->derr, 0x02, 1, st)) != hipSuccess)
                return hip_fail(probs[i], e, "error word");
        if ((e = launch_sweep_group_table(L.path, L.mt, L.cbw, L.mh, dtab + offs[li], L.nwg, L.lds, st)) !=
            hipSuccess)
            return hip_fail(nullptr, e, "group table launch");
        for (int i : L.members) {
            phia_problem* p = probs[i];
            const int iters = (p->geo.nblocks + p->geo.ngroups - 1) / p->geo.ngroups;
            p->seq += static_cast<uint32_t>(iters) * static_cast<uint32_t>(k_end[i] - p->k + 1);
            p->k = k_end[i];
            p->has_run = true;
        }
    }
    for (int i : alone) {
        phia_status s2 = phia_anneal_run(probs[i], k_end[i]);
        if (s2 != PHIA_OK) return s2;
    }
    return PHIA_OK;
}

}  // namespace phia

// ----------------------------------------------------------- batch plan --
// A batch plan owns the replica state of its problems and one instantiated
// HIP graph that runs every problem's whole anneal: a reset of the work
// queue, the persistent sweep over the instances it holds (couplings that are
// all FP4 integers, N <= 512, no accept/reject step), then, for the other
// instances, an init kernel and one sweep kernel per bucket of similar
// instances.  Seeds live in device memory and are refreshed before each
// launch, so the graph is built once and launched many times.
struct phia_batch {
    int dev = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    std::vector<phia_problem*> probs;
    std::vector<int64_t> steps;
    // persistent sweep
    BatchInst* dinst = nullptr;
    BatchItem* ditems = nullptr;
    int nitems = 0;
    int* dqueue = nullptr;
    size_t fp4_lds = 0;
    int n_fp4 = 0;
    // one-item-per-workgroup sweep of the remaining instances
    SweepArgs* dtab = nullptr;
    // seeds: pinned host staging copy and device array
    uint64_t* hseeds = nullptr;
    uint64_t* dseeds = nullptr;
    hipEvent_t seed_ev = nullptr;
    bool seed_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool launched = false;
    bool broken = false;  // a member problem was destroyed
};

namespace phia {

// Wait for the batch's work (results of its problems are read after it).
hipError_t batch_wait(phia_batch* b)
{
    if (!b || !b->launched) return hipSuccess;
    hipError_t e = hipStreamSynchronize(b->st);
    if (e == hipSuccess) b->launched = false;
    return e;
}

// A member problem is being destroyed: wait for the batch and drop it.
void batch_forget(phia_batch* b, phia_problem* p)
{
    if (!b) return;
    (void)batch_wait(b);
    for (phia_problem*& q : b->probs)
        if (q == p) q = nullptr;
    b->broken = true;
}

}  // namespace phia

namespace {

// Instances the persistent sweep takes: int8 path with FP4 operand
// couplings, N <= 512, no accept/reject step, and every row energy sum (and
// partial sum) below 2^24 in magnitude, so that the sweep's FP32 sums are
// exact: |sum_i s_i (I_i + h_i)| <= N (maxrow + max |h|) <= 2 maxrow N.
bool fp4_batchable(const phia_problem* p)
{
    return p->path == PHIA_PATH_I8 && p->has_j4 && p->Np <= kBatchFp4MaxNp && !p->mh &&
           2 * p->maxrow * static_cast<int64_t>(p->N) < (int64_t(1) << 24);
}

void release(phia_batch* b)
{
    if (!b) return;
    (void)hipSetDevice(b->dev);
    if (b->launched && b->st) (void)hipStreamSynchronize(b->st);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dinst) (void)hipFree(b->dinst);
    if (b->ditems) (void)hipFree(b->ditems);
    if (b->dqueue) (void)hipFree(b->dqueue);
    if (b->dtab) (void)hipFree(b->dtab);
    if (b->dseeds) (void)hipFree(b->dseeds);
    if (b->hseeds) (void)hipHostFree(b->hseeds);
    if (b->seed_ev) (void)hipEventDestroy(b->seed_ev);
    for (phia_problem* p : b->probs)
        if (p && p->batch == b) p->batch = nullptr;
    if (b->own_stream && b->st) (void)hipStreamDestroy(b->st);
    delete b;
}

}  // namespace

extern "C" {

phia_status phia_batch_create(phia_problem* const* probs, int32_t count, const int32_t* replicas,
                              const int64_t* steps, const phia_schedule* scheds, phia_batch** out)
{
    clear_error();
    if (!out) return fail(PHIA_EINVAL, "out is null");
    *out = nullptr;
    if (!probs || !replicas || !steps || !scheds) return fail(PHIA_EINVAL, "null argument");
    if (count < 1 || count > (1 << 22)) return fail(PHIA_EINVAL, "count = %d out of range", count);
    const int dev = probs[0] ? probs[0]->dev : 0;
    for (int i = 0; i < count; ++i) {
        phia_problem* p = probs[i];
        phia_status st = check_usable(p);
        if (st != PHIA_OK) return st;
        if (p->batch) return fail(PHIA_ESTATE, "problem %d already belongs to a batch", i);
        if (p->dev != dev) return fail(PHIA_EINVAL, "problem %d is on another device", i);
        if (p->path != PHIA_PATH_I8 && p->path != PHIA_PATH_BF16HILO)
            return fail(PHIA_EINVAL, "problem %d uses the %s path; batches run I8/BF16HILO", i,
                        p->path == PHIA_PATH_FP32 ? "FP32" : "ELL");
        if (p->Np > kBatchMaxNp) return fail(PHIA_ERANGE, "problem %d: N = %d exceeds %d for batches", i, p->N, kBatchMaxNp);
        if ((st = check_schedule(replicas[i], steps[i], &scheds[i])) != PHIA_OK) return st;
        if (scheds[i].initial_kick) return fail(PHIA_EINVAL, "schedule %d: batches run without the initial kick", i);
        if (steps[i] >= (int64_t(1) << 31)) return fail(PHIA_EINVAL, "problem %d: too many steps", i);
    }
    {
        std::vector<const phia_problem*> sorted(probs, probs + count);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(PHIA_EINVAL, "a problem appears twice in the batch");
    }
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(nullptr, e, "synchronise");

    phia_batch* b = new (std::nothrow) phia_batch();
    if (!b) return fail(PHIA_ENOMEM, "host allocation failed");
    b->dev = dev;
    b->probs.assign(probs, probs + count);
    b->steps.assign(steps, steps + count);
    // Stream capture needs a stream other than the null stream.
    b->st = probs[0]->st;
    if (!b->st) {
        if ((e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking)) != hipSuccess) {
            delete b;
            return hip_fail(nullptr, e, "stream creation");
        }
        b->own_stream = true;
    }
    auto bail = [&](phia_status st_) {
        release(b);
        return st_;
    };
    if ((e = hipMalloc(&b->dseeds, sizeof(uint64_t) * count)) != hipSuccess ||
        (e = hipHostMalloc(&b->hseeds, sizeof(uint64_t) * count, hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->seed_ev, hipEventDisableTiming)) != hipSuccess)
        return bail(fail(PHIA_ENOMEM, "seed buffers: %s", hipGetErrorString(e)));
    for (int i = 0; i < count; ++i) b->hseeds[i] = 0;

    // Replica state and schedules of every problem (host tables kept until
    // the device has copied them).
    std::vector<std::vector<float>> ctabs(static_cast<size_t>(count));
    std::vector<BatchInst> insts;
    std::vector<BatchItem> items;
    std::vector<int64_t> item_cost;
    std::vector<SweepArgs> init_tab;
    std::map<std::tuple<int, int, int, int>, Bucket> buckets;
    for (int i = 0; i < count; ++i) {
        phia_problem* p = probs[i];
        kick_factors(p, steps[i], &scheds[i], ctabs[i]);
        bool reuse = false;
        phia_status st_ = make_resident(p);
        if (st_ == PHIA_OK) st_ = setup_state(p, replicas[i], steps[i], &scheds[i], 0, ctabs[i], reuse, false);
        if (st_ != PHIA_OK) return bail(st_);
        p->batch = b;
        p->geo = Geometry{};
        p->geo.ok = true;
        p->geo.G = 1;
        p->geo.j_lds = 1;
        if (fp4_batchable(p)) {
            p->geo.kind = 3;
            p->geo.mt = 2;
            p->geo.rows = kBatchRows;
            p->geo.nblocks = (replicas[i] + kBatchRows - 1) / kBatchRows;
            p->geo.ngroups = p->geo.nblocks;
            BatchInst a{};
            a.J4 = static_cast<const unsigned char*>(p->dJ4);
            a.h = p->dh;
            a.ctab = p->dctab;
            a.seed = b->dseeds + i;
            a.x = p->dx;
            a.v = p->dv;
            a.bestE = p->dbestE;
            a.bestS = p->dbestS;
            a.bestStep = p->dbestStep;
            a.k0 = 0;
            a.k1 = steps[i];
            a.L = p->L;
            a.eps = p->eps;
            a.gamma = p->gamma;
            a.N = p->N;
            a.Np = p->Np;
            a.R = replicas[i];
            a.deriv = p->deriv;
            a.init = 1;
            const bool dbl = batch_fp4_lds_bytes(p->Np, true) <= static_cast<size_t>(kLdsMax);
            b->fp4_lds = std::max(b->fp4_lds, batch_fp4_lds_bytes(p->Np, dbl));
            for (int blk = 0; blk < p->geo.nblocks; ++blk) {
                items.push_back(BatchItem{static_cast<int32_t>(insts.size()), blk});
                const int rows = std::min(kBatchRows, replicas[i] - blk * kBatchRows);
                item_cost.push_back(static_cast<int64_t>(p->Np) * steps[i] * (rows > 16 ? 2 : 1));
            }
            insts.push_back(a);
            continue;
        }
        p->geo.mt = 1;
        p->geo.rows = 16;
        p->geo.nblocks = (replicas[i] + 15) / 16;
        p->geo.ngroups = p->geo.nblocks;
        const int ncb = p->Np / 16;
        const int cbw = ncb <= kWaves * 2 ? 2 : 4;
        const int jl = sweep_batch_lds_bytes(p->path, p->Np, 1, p->mh) <= static_cast<size_t>(kLdsMax) ? 1 : 0;
        p->geo.cbw = cbw;
        p->geo.j_lds = jl;
        if ((st_ = setup_mh_geometry(p)) != PHIA_OK) return bail(st_);
        SweepArgs a = sweep_args(p);
        a.inc = 0;  // table launches carry no flip-incremental variant
        a.J = p->dJ;
        a.k0 = 0;
        a.k1 = steps[i];
        a.etrace = nullptr;
        a.G = 1;
        a.ncb = ncb;
        a.rows = 16;
        a.j_lds = jl;
        a.seedp = b->dseeds + i;
        init_tab.push_back(a);
        Bucket& bk = buckets[std::make_tuple(p->path, cbw, jl, p->mh)];
        bk.path = p->path;
        bk.cbw = cbw;
        bk.jl = jl;
        bk.mh = p->mh;
        bk.lds = std::max(bk.lds, sweep_batch_lds_bytes(p->path, p->Np, jl, p->mh));
        for (int blk = 0; blk < p->geo.nblocks; ++blk) {
            SweepArgs it = a;
            it.block = blk;
            it.nblocks = blk + 1;
            it.ngroups = 1;
            bk.items.push_back(it);
        }
    }
    b->n_fp4 = static_cast<int>(insts.size());
    // Persistent sweep items: costliest first, so that the queue's tail holds
    // the shortest items.
    {
        std::vector<size_t> ord(items.size());
        for (size_t t = 0; t < ord.size(); ++t) ord[t] = t;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t u, size_t w) { return item_cost[u] > item_cost[w]; });
        std::vector<BatchItem> sorted;
        sorted.reserve(items.size());
        for (size_t t : ord) sorted.push_back(items[t]);
        items.swap(sorted);
    }
    b->nitems = static_cast<int>(items.size());
    if (!items.empty()) {
        if ((e = hipMalloc(&b->dinst, sizeof(BatchInst) * insts.size())) != hipSuccess ||
            (e = hipMalloc(&b->ditems, sizeof(BatchItem) * items.size())) != hipSuccess ||
            (e = hipMalloc(&b->dqueue, 256)) != hipSuccess)
            return bail(fail(PHIA_ENOMEM, "work table allocation failed"));
        if ((e = hipMemcpy(b->dinst, insts.data(), sizeof(BatchInst) * insts.size(), hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(b->ditems, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice)) !=
                hipSuccess)
            return bail(hip_fail(nullptr, e, "work table upload"));
    }
    // One device table for the remaining instances: init entries, then every
    // bucket's items.
    std::vector<SweepArgs> host_tab(init_tab);
    std::vector<size_t> offs;
    for (auto& kv : buckets) {
        order_items(kv.second.items);
        offs.push_back(host_tab.size());
        host_tab.insert(host_tab.end(), kv.second.items.begin(), kv.second.items.end());
    }
    if (!host_tab.empty()) {
        if ((e = hipMalloc(&b->dtab, sizeof(SweepArgs) * host_tab.size())) != hipSuccess)
            return bail(fail(PHIA_ENOMEM, "work table allocation failed"));
        if ((e = hipMemcpy(b->dtab, host_tab.data(), sizeof(SweepArgs) * host_tab.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return bail(hip_fail(nullptr, e, "work table upload"));
        for (auto& kv : buckets)
            if ((e = prepare_sweep_batch(kv.second.path, kv.second.cbw, kv.second.mh, kv.second.lds)) != hipSuccess)
                return bail(hip_fail(nullptr, e, "kernel attributes"));
    }
    if (b->nitems > 0 && batch_fp4_grid(b->fp4_lds) < 1)
        return bail(fail(PHIA_EDEVICE, "the persistent batch sweep does not fit the device"));
    // schedules and state set-up above ran on the problems' streams
    if ((e = hipDeviceSynchronize()) != hipSuccess) return bail(hip_fail(nullptr, e, "state set-up"));

    if ((e = hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return bail(hip_fail(nullptr, e, "graph capture"));
    hipError_t le = hipSuccess;
    if (b->nitems > 0) {
        le = launch_batch_queue_reset(b->dqueue, b->st);
        if (le == hipSuccess) le = launch_batch_fp4(b->dinst, b->ditems, b->nitems, b->dqueue, b->fp4_lds, b->st);
    }
    if (le == hipSuccess && !init_tab.empty()) le = launch_init_batch(b->dtab, static_cast<int>(init_tab.size()), b->st);
    size_t bi = 0;
    for (auto& kv : buckets) {
        if (le == hipSuccess)
            le = launch_sweep_batch(kv.second.path, kv.second.cbw, kv.second.mh, b->dtab + offs[bi],
                                    static_cast<int>(kv.second.items.size()), kv.second.lds, b->st);
        ++bi;
    }
    e = hipStreamEndCapture(b->st, &b->graph);
    if (le != hipSuccess || e != hipSuccess)
        return bail(hip_fail(nullptr, le != hipSuccess ? le : e, "graph capture of the batch"));
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
        return bail(hip_fail(nullptr, e, "graph instantiation"));
    for (int i = 0; i < count; ++i) {
        probs[i]->k = 0;
        probs[i]->started = false;
        probs[i]->has_run = false;
    }
    *out = b;
    return PHIA_OK;
}

phia_status phia_batch_launch(phia_batch* b, const uint64_t* seeds)
{
    clear_error();
    if (!b || !seeds) return fail(PHIA_EINVAL, "null argument");
    hipError_t e = hipSetDevice(b->dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    if (b->broken) return fail(PHIA_ESTATE, "a problem of the batch has been destroyed");
    for (phia_problem* p : b->probs)
        if (p->poisoned) return fail(PHIA_EDEVICE, "a problem of the batch is poisoned");
    // the staging copy of the previous launch has been read before it is rewritten
    if (b->seed_pending && (e = hipEventSynchronize(b->seed_ev)) != hipSuccess)
        return hip_fail(nullptr, e, "seed staging");
    const size_t n = b->probs.size();
    for (size_t i = 0; i < n; ++i) b->hseeds[i] = seeds[i];
    if ((e = hipMemcpyAsync(b->dseeds, b->hseeds, sizeof(uint64_t) * n, hipMemcpyHostToDevice, b->st)) !=
            hipSuccess ||
        (e = hipEventRecord(b->seed_ev, b->st)) != hipSuccess)
        return hip_fail(nullptr, e, "seed upload");
    b->seed_pending = true;
    if ((e = hipGraphLaunch(b->exec, b->st)) != hipSuccess) {
        for (phia_problem* p : b->probs) p->poisoned = true;
        return hip_fail(nullptr, e, "batch graph launch");
    }
    b->launched = true;
    for (size_t i = 0; i < n; ++i) {
        phia_problem* p = b->probs[i];
        p->seed = seeds[i];
        p->k = b->steps[i];
        p->started = true;
        p->has_run = true;
    }
    return PHIA_OK;
}

phia_status phia_batch_sync(phia_batch* b)
{
    clear_error();
    if (!b) return fail(PHIA_EINVAL, "null argument");
    hipError_t e = hipSetDevice(b->dev);
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) {
        for (phia_problem* p : b->probs)
            if (p) p->poisoned = true;
        return hip_fail(nullptr, e, "batch");
    }
    b->launched = false;
    return PHIA_OK;
}

void phia_batch_destroy(phia_batch* b) { release(b); }

phia_status phia_batch_run(phia_problem* const* probs, int32_t count, const int32_t* replicas, const int64_t* steps,
                           const phia_schedule* scheds, const uint64_t* seeds)
{
    clear_error();
    if (!seeds) return fail(PHIA_EINVAL, "null argument");
    phia_batch* b = nullptr;
    phia_status st = phia_batch_create(probs, count, replicas, steps, scheds, &b);
    if (st != PHIA_OK) return st;
    st = phia_batch_launch(b, seeds);
    if (st == PHIA_OK) st = phia_batch_sync(b);
    release(b);
    return st;
}

}  // extern "C"
