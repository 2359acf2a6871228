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

extern "C" phia_status phia_batch_run(phia_problem* const* probs, int32_t count, const int32_t* replicas,
                                      const int64_t* steps, const phia_schedule* scheds, const uint64_t* seeds)
{
    clear_error();
    if (!probs || !replicas || !steps || !scheds || !seeds) return fail(PHIA_EINVAL, "null argument");
    if (count < 1 || count > (1 << 22)) return fail(PHIA_EINVAL, "count = %d out of range", count);
    const int dev = probs[0] ? probs[0]->dev : 0;
    for (int i = 0; i < count; ++i) {
        phia_problem* p = probs[i];
        phia_status st = check_usable(p);
        if (st != PHIA_OK) return st;
        if (p->dev != dev) return fail(PHIA_EINVAL, "problem %d is on another device", i);
        if (p->path == PHIA_PATH_FP32) return fail(PHIA_EINVAL, "problem %d uses the FP32 path; batches run I8/BF16HILO", i);
        if (p->Np > kBatchMaxNp) return fail(PHIA_ERANGE, "problem %d: N = %d exceeds %d for batches", i, p->N, kBatchMaxNp);
        if ((st = check_schedule(replicas[i], steps[i], &scheds[i])) != PHIA_OK) return st;
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

    // Stream capture needs a stream other than the null stream.
    hipStream_t st = probs[0]->st;
    bool own_stream = false;
    if (!st) {
        if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(nullptr, e, "stream creation");
        own_stream = true;
    }
    std::vector<hipStream_t> saved(static_cast<size_t>(count));
    for (int i = 0; i < count; ++i) {
        saved[i] = probs[i]->st;
        probs[i]->st = st;
    }
    auto restore = [&]() {
        for (int i = 0; i < count; ++i) probs[i]->st = saved[i];
        if (own_stream) (void)hipStreamDestroy(st);
    };

    // Replica state and schedules (host tables stay alive until the final sync).
    std::vector<std::vector<float>> ctabs(static_cast<size_t>(count));
    std::vector<SweepArgs> init_tab(static_cast<size_t>(count));
    std::map<std::tuple<int, int, int, int>, Bucket> buckets;
    phia_status st_ = PHIA_OK;
    for (int i = 0; i < count && st_ == PHIA_OK; ++i) {
        phia_problem* p = probs[i];
        kick_factors(p, steps[i], &scheds[i], ctabs[i]);
        bool reuse = false;
        st_ = setup_state(p, replicas[i], steps[i], &scheds[i], seeds[i], ctabs[i], reuse, false);
        if (st_ != PHIA_OK) break;
        p->geo = Geometry{};
        p->geo.ok = true;
        p->geo.mt = 1;
        p->geo.G = 1;
        p->geo.rows = 16;
        p->geo.nblocks = (replicas[i] + 15) / 16;
        p->geo.ngroups = p->geo.nblocks;
        const int ncb = p->Np / 16;
        const int cbw = ncb <= kWaves * 2 ? 2 : 4;
        const int jl = sweep_batch_lds_bytes(p->path, p->Np, 1, p->mh) <= static_cast<size_t>(kLdsMax) ? 1 : 0;
        p->geo.cbw = cbw;
        p->geo.j_lds = jl;
        if ((st_ = setup_mh_geometry(p)) != PHIA_OK) break;
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
        init_tab[static_cast<size_t>(i)] = a;
        Bucket& b = buckets[std::make_tuple(p->path, cbw, jl, p->mh)];
        b.path = p->path;
        b.cbw = cbw;
        b.jl = jl;
        b.mh = p->mh;
        b.lds = std::max(b.lds, sweep_batch_lds_bytes(p->path, p->Np, jl, p->mh));
        for (int blk = 0; blk < p->geo.nblocks; ++blk) {
            SweepArgs it = a;
            it.block = blk;
            it.nblocks = blk + 1;
            it.ngroups = 1;
            b.items.push_back(it);
        }
    }
    if (st_ != PHIA_OK) {
        restore();
        return st_;
    }
    size_t total_items = 0;
    for (auto& kv : buckets) {
        order_items(kv.second.items);
        total_items += kv.second.items.size();
    }
    // One device table: the init entries, then every bucket's items.
    std::vector<SweepArgs> host_tab(init_tab);
    std::vector<size_t> offs;
    for (auto& kv : buckets) {
        offs.push_back(host_tab.size());
        host_tab.insert(host_tab.end(), kv.second.items.begin(), kv.second.items.end());
    }
    SweepArgs* dtab = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if ((e = hipMalloc(&dtab, sizeof(SweepArgs) * host_tab.size())) != hipSuccess) {
        restore();
        return fail(PHIA_ENOMEM, "work table allocation failed");
    }
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipFree(dtab);
        restore();
    };
    if ((e = hipMemcpyAsync(dtab, host_tab.data(), sizeof(SweepArgs) * host_tab.size(), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        cleanup();
        return hip_fail(nullptr, e, "work table upload");
    }
    for (auto& kv : buckets)
        if ((e = prepare_sweep_batch(kv.second.path, kv.second.cbw, kv.second.mh, kv.second.lds)) != hipSuccess) {
            cleanup();
            return hip_fail(nullptr, e, "kernel attributes");
        }
    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        cleanup();
        return hip_fail(nullptr, e, "graph capture");
    }
    hipError_t le = launch_init_batch(dtab, count, st);
    size_t bi = 0;
    for (auto& kv : buckets) {
        if (le == hipSuccess)
            le = launch_sweep_batch(kv.second.path, kv.second.cbw, kv.second.mh, dtab + offs[bi],
                                    static_cast<int>(kv.second.items.size()), kv.second.lds, st);
        ++bi;
    }
    e = hipStreamEndCapture(st, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        cleanup();
        return hip_fail(nullptr, le != hipSuccess ? le : e, "graph capture of the batch");
    }
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess ||
        (e = hipGraphLaunch(exec, st)) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess) {
        for (int i = 0; i < count; ++i) probs[i]->poisoned = true;
        cleanup();
        return hip_fail(nullptr, e, "batch graph");
    }
    cleanup();
    for (int i = 0; i < count; ++i) {
        probs[i]->k = steps[i];
        probs[i]->started = true;
        probs[i]->has_run = true;
    }
    (void)total_items;
    return PHIA_OK;
}
