// Graph-captured form of the batched single-angle-pair scan (Eq. (5) over
// instances x (beta, gamma) grids, App. C's level space), with optional
// statevector work items on cells of the same grid.
//
// Creating a plan does the per-instance work once: the occupied levels and
// weights are compacted and uploaded, every bucket's launch shape is chosen
// (tuned on the real queue), and the launches are captured in one HIP graph
// with one parallel branch per scan bucket and one per group of statevector
// items (one group per n), so both paths go out with a single hipGraphLaunch. A run
// then uploads only the angle grid and the items' angles (one copy from
// pinned staging) and replays the graph. Every queue counter is cleared by a
// kernel inside the graph, so the graph holds kernel nodes only.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "stream_pool.h"

namespace gqaoa {

struct ScanPlan {
    int device = -1;
    int num_inst = 0, nb = 0, ng = 0, per_inst = 0, num_items = 0;
    size_t n_b = 0, n_g = 0;           // angle counts (nb or num_inst*nb, likewise ng)
    std::vector<int32_t> item_cell;    // launch order: [k][2] = gamma index, beta index
    std::vector<int32_t> item_inst;    // launch order: instance
    std::vector<int32_t> item_out;     // launch order: caller's item index
    char *dev = nullptr;               // device block: dynamic region first, then the static tables
    char *stage = nullptr;             // pinned mirror of the dynamic region
    size_t dyn_bytes = 0;
    size_t off_b = 0, off_g = 0, off_items = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> branch;   // one per scan bucket, then one per item group
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;      // one per branch
    hipEvent_t staged = nullptr;       // the last upload has read the staging
    hipEvent_t done = nullptr;         // the last replay has finished
};

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Item angles in launch order, from the grid held in the staging block.
static void fill_items(ScanPlan *P) {
    const double *b = reinterpret_cast<const double *>(P->stage + P->off_b);
    const double *g = reinterpret_cast<const double *>(P->stage + P->off_g);
    SvItem *it = reinterpret_cast<SvItem *>(P->stage + P->off_items);
    for (int k = 0; k < P->num_items; ++k) {
        const int i = P->item_inst[k];
        const size_t bo = P->per_inst ? (size_t)i * P->nb : 0, go = P->per_inst ? (size_t)i * P->ng : 0;
        it[k] = SvItem{i, P->item_out[k], b[bo + P->item_cell[2 * k + 1]], g[go + P->item_cell[2 * k]]};
    }
}

static void release(ScanPlan *P) {
    if (!P) return;
    if (P->done) (void)hipEventSynchronize(P->done);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->fork) (void)hipEventDestroy(P->fork);
    for (hipEvent_t e : P->join) (void)hipEventDestroy(e);
    if (P->staged) (void)hipEventDestroy(P->staged);
    if (P->done) (void)hipEventDestroy(P->done);
    // the capture and branch streams go back to the pool once the plan was
    // instantiated (every capture on them has ended); a plan that failed
    // half-way destroys them
    std::vector<hipStream_t> ss(P->branch);
    if (P->cap) ss.push_back(P->cap);
    if (P->exec) {
        stream_pool_give(P->device, ss);
    } else {
        for (hipStream_t x : ss) (void)hipStreamDestroy(x);
    }
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->dev) (void)hipFree(P->dev);
    if (P->stage) (void)hipHostFree(P->stage);
    delete P;
}

// Owns a plan under construction; frees it, after the work already
// enqueued on the creating stream, unless released to the caller.
struct PlanGuard {
    ScanPlan *p;
    hipStream_t st;
    ~PlanGuard() {
        if (!p) return;
        (void)hipStreamSynchronize(st);
        release(p);
    }
};

// Enqueues every launch of the plan, each scan bucket and each group of
// items (one n) on a branch of its own, forked from and joined back to
// `cap`: they are independent, so the tail of one overlaps the others.
static int enqueue_all(ScanPlan *P, const DeviceInfo &dev, const std::vector<ScanArgs> &bucket_args,
                       const std::vector<int> &bucket_ids, const std::vector<TileChoice> &tiles,
                       unsigned int *counters, const std::vector<SvItemsArgs> &item_args) {
    int s;
    GQ_HIP(hipEventRecord(P->fork, P->cap));
    for (size_t q = 0; q < bucket_args.size(); ++q) {
        GQ_HIP(hipStreamWaitEvent(P->branch[q], P->fork, 0));
        if ((s = scan_launch_bucket(bucket_ids[q], tiles[q], dev, bucket_args[q], counters + bucket_ids[q],
                                    P->branch[q])))
            return s;
    }
    for (size_t q = 0; q < item_args.size(); ++q) {
        hipStream_t side = P->branch[bucket_args.size() + q];
        GQ_HIP(hipStreamWaitEvent(side, P->fork, 0));
        if ((s = sv_items_launch(item_args[q], dev, side))) return s;
    }
    for (size_t q = 0; q < P->branch.size(); ++q) {
        GQ_HIP(hipEventRecord(P->join[q], P->branch[q]));
        GQ_HIP(hipStreamWaitEvent(P->cap, P->join[q], 0));
    }
    return GQAOA_OK;
}

int scan_plan_create(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists,
                     int hist_stride, const int32_t *target_host, int nb, const double *betas, int ng,
                     const double *gammas, int per_inst, int num_p, const int32_t *p_list, float *psol,
                     float *energy, const int32_t *tile, int num_items, const int32_t *items,
                     const uint8_t *costs, const uint64_t *cost_off, float *item_psol, float *item_energy,
                     hipStream_t st, ScanPlan **out) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    ScanHost H;
    if ((s = scan_host_tables(num_inst, n_host, m_host, hists, hist_stride, target_host, nullptr, p_list[num_p - 1],
                              &H)))
        return s;
    std::vector<int32_t> item_inst(num_items);
    for (int k = 0; k < num_items; ++k) item_inst[k] = items[3 * k];
    ItemOrder ord;
    if (num_items && (s = sv_items_order(n_host, num_items, item_inst.data(), dev, &ord))) return s;

    PlanGuard G{new (std::nothrow) ScanPlan, st};
    if (!G.p) return fail(GQAOA_EINVAL, "out of host memory");
    ScanPlan *P = G.p;
    P->device = dev.device;
    P->num_inst = num_inst;
    P->nb = nb;
    P->ng = ng;
    P->per_inst = per_inst;
    P->num_items = num_items;
    P->n_b = (size_t)nb * (per_inst ? num_inst : 1);
    P->n_g = (size_t)ng * (per_inst ? num_inst : 1);
    P->item_cell.resize(2 * (size_t)num_items);
    P->item_inst.resize(num_items);
    P->item_out.resize(num_items);
    for (int k = 0; k < num_items; ++k) {
        const int o = ord.order[k];
        P->item_inst[k] = items[3 * o];
        P->item_cell[2 * k] = items[3 * o + 1];
        P->item_cell[2 * k + 1] = items[3 * o + 2];
        P->item_out[k] = o;
    }

    // device block: [betas | gammas | items] (rewritten by runs), then
    // [slots | lev | w | counters | cost offsets | m | target]
    P->off_b = 0;
    P->off_g = al256(8 * P->n_b);
    P->off_items = P->off_g + al256(8 * P->n_g);
    P->dyn_bytes = P->off_items + al256(sizeof(SvItem) * (size_t)num_items);
    const size_t o_slots = P->dyn_bytes;
    const size_t o_lev = o_slots + al256(sizeof(ScanSlot) * H.slots.size());
    const size_t o_w = o_lev + al256(4 * std::max<size_t>(1, H.lev.size()));
    const size_t o_cnt = o_w + al256(4 * std::max<size_t>(1, H.w.size()));
    const size_t o_coff = o_cnt + al256(4 * (size_t)scan_num_buckets());
    const size_t o_m = o_coff + al256(8 * (size_t)num_inst);
    const size_t o_t = o_m + al256(4 * (size_t)num_inst);
    const size_t total = o_t + al256(4 * (size_t)num_inst);
    GQ_HIP(hipMalloc(&P->dev, total));
    GQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&P->stage), std::max<size_t>(P->dyn_bytes, 256), hipHostMallocDefault));
    GQ_HIP(hipEventCreateWithFlags(&P->fork, hipEventDisableTiming));
    GQ_HIP(hipEventCreateWithFlags(&P->staged, hipEventDisableTiming));
    GQ_HIP(hipEventCreateWithFlags(&P->done, hipEventDisableTiming));
    {
        std::vector<hipStream_t> c;
        const int sc = stream_pool_take(1, &c);
        if (!c.empty()) P->cap = c[0];
        if (sc) return sc;
    }

    // static tables and the first grid
    std::memcpy(P->stage + P->off_b, betas, 8 * P->n_b);
    std::memcpy(P->stage + P->off_g, gammas, 8 * P->n_g);
    fill_items(P);
    std::vector<int32_t> tg(num_inst, 0);
    if (target_host) tg.assign(target_host, target_host + num_inst);
    std::vector<uint64_t> coff(num_inst, 0);
    if (num_items)
        for (int i = 0; i < num_inst; ++i) coff[i] = cost_off[i];
    GQ_HIP(hipMemcpyAsync(P->dev, P->stage, P->dyn_bytes, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(P->dev + o_slots, H.slots.data(), sizeof(ScanSlot) * H.slots.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(P->dev + o_lev, H.lev.data(), 4 * H.lev.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(P->dev + o_w, H.w.data(), 4 * H.w.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(P->dev + o_coff, coff.data(), 8 * (size_t)num_inst, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(P->dev + o_m, m_host, 4 * (size_t)num_inst, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(P->dev + o_t, tg.data(), 4 * (size_t)num_inst, hipMemcpyHostToDevice, st));

    // per-bucket launch arguments and shapes (tuned on the caller's stream)
    unsigned int *counters = reinterpret_cast<unsigned int *>(P->dev + o_cnt);
    ScanArgs a{};
    a.lev = reinterpret_cast<const int32_t *>(P->dev + o_lev);
    a.w = reinterpret_cast<const float *>(P->dev + o_w);
    a.betas = reinterpret_cast<const double *>(P->dev + P->off_b);
    a.gammas = reinterpret_cast<const double *>(P->dev + P->off_g);
    a.psol = psol;
    a.energy = energy;
    a.nb = nb;
    a.ng = ng;
    a.ntiles = (nb + 63) / 64;
    a.num_p = num_p;
    a.per_inst = per_inst;
    for (int q = 0; q < num_p; ++q) a.p_list[q] = p_list[q];
    std::vector<ScanArgs> bucket_args;
    std::vector<int> bucket_ids;
    std::vector<TileChoice> tiles;
    for (int bk = 0; bk < scan_num_buckets(); ++bk) {
        const int nslots = H.bucket_first[bk + 1] - H.bucket_first[bk];
        if (!nslots) continue;
        ScanArgs ab = a;
        ab.slots = reinterpret_cast<const ScanSlot *>(P->dev + o_slots) + H.bucket_first[bk];
        ab.total_items = (unsigned)nslots * (unsigned)ng * (unsigned)ab.ntiles;
        TileChoice tc;
        if ((s = scan_choose_tile(bk, dev, ab, counters + bk, tile, st, &tc))) return s;
        bucket_args.push_back(ab);
        bucket_ids.push_back(bk);
        tiles.push_back(tc);
    }
    std::vector<SvItemsArgs> item_args;
    for (size_t gi = 0; gi + 1 < ord.first.size(); ++gi) {
        const int k0 = ord.first[gi], k1 = ord.first[gi + 1];
        SvItemsArgs ia{};
        ia.items = reinterpret_cast<const SvItem *>(P->dev + P->off_items) + k0;
        ia.num_items = k1 - k0;
        ia.n = n_host[P->item_inst[k0]];
        ia.costs = costs;
        ia.cost_off = reinterpret_cast<const uint64_t *>(P->dev + o_coff);
        ia.m = reinterpret_cast<const int32_t *>(P->dev + o_m);
        ia.target = reinterpret_cast<const int32_t *>(P->dev + o_t);
        ia.num_p = num_p;
        for (int q = 0; q < num_p; ++q) ia.p_list[q] = p_list[q];
        ia.psol = item_psol;
        ia.energy = item_energy;
        item_args.push_back(ia);
    }
    GQ_HIP(hipStreamSynchronize(st));  // uploads and tuning done; host tables end here
    const size_t nbranch = bucket_args.size() + item_args.size();
    if ((s = stream_pool_take(nbranch, &P->branch))) return s;
    for (size_t q = 0; q < nbranch; ++q) {
        hipEvent_t e = nullptr;
        GQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        P->join.push_back(e);
    }

    // capture: one branch per path
    GQ_HIP(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
    s = enqueue_all(P, dev, bucket_args, bucket_ids, tiles, counters, item_args);
    hipGraph_t graph = nullptr;
    const hipError_t e_end = hipStreamEndCapture(P->cap, &graph);
    P->graph = graph;
    if (s) return s;
    GQ_HIP(e_end);
    GQ_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
    GQ_HIP(hipEventRecord(P->staged, st));
    GQ_HIP(hipEventRecord(P->done, st));
    *out = P;
    G.p = nullptr;
    return GQAOA_OK;
}

int scan_plan_run(ScanPlan *P, const double *betas, const double *gammas, hipStream_t st) {
    int cur = -1;
    GQ_HIP(hipGetDevice(&cur));
    if (cur != P->device) return fail(GQAOA_EINVAL, "plan made on device %d, current device is %d", P->device, cur);
    if (betas)
        for (size_t k = 0; k < std::max(P->n_b, P->n_g); ++k)
            if ((k < P->n_b && !std::isfinite(betas[k])) || (k < P->n_g && !std::isfinite(gammas[k])))
                return fail(GQAOA_EINVAL, "non-finite angle in the grid");
    GQ_HIP(hipStreamWaitEvent(st, P->done, 0));  // the previous replay has read the device grid
    if (betas) {
        GQ_HIP(hipEventSynchronize(P->staged));  // the previous upload has read the staging
        std::memcpy(P->stage + P->off_b, betas, 8 * P->n_b);
        std::memcpy(P->stage + P->off_g, gammas, 8 * P->n_g);
        fill_items(P);
        GQ_HIP(hipMemcpyAsync(P->dev, P->stage, P->dyn_bytes, hipMemcpyHostToDevice, st));
        GQ_HIP(hipEventRecord(P->staged, st));
    }
    GQ_HIP(hipGraphLaunch(P->exec, st));
    GQ_HIP(hipEventRecord(P->done, st));
    return GQAOA_OK;
}

void scan_plan_destroy(ScanPlan *P) { release(P); }

}  // namespace gqaoa
