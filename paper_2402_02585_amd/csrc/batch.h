// Launch pieces of the batched single-angle-pair scan (hist.hip) and of its
// statevector work items (sv_items.hip), shared by the eager entry points and
// by the graph-captured scan plan (plan.hip).
#pragma once

#include <vector>

#include "internal.h"
#include "tune_cache.h"

namespace gqaoa {

// ---- level-space scan ------------------------------------------------------------------
constexpr int kScanMaxP = 16;

struct ScanSlot {          // one instance inside a bucket, in queue order
    int32_t inst;          // caller's instance index
    int32_t lev_off;       // into lev/w
    int32_t K;             // occupied levels
    int32_t t_idx;         // 0 when the target level is occupied (it comes first among them), else -1
    int32_t pmax;          // rounds to run for this instance
    int32_t pad[3];
};

struct ScanArgs {
    const ScanSlot *slots;
    const int32_t *lev;
    const float *w;
    const double *betas;
    const double *gammas;
    float *psol;
    float *energy;
    int32_t *first_p;      // crossing mode: [inst][ng][nb] first round with P >= threshold (0: none)
    float threshold;
    unsigned int *counter;
    unsigned int total_items;
    int nb, ng, ntiles, num_p;
    int per_inst;          // angle grids are per instance
    int p_list[kScanMaxP];
};

// Host tables of a scan: occupied levels and weights of every instance,
// compacted, and one slot per instance, grouped by bucket (slots
// [bucket_first[b], bucket_first[b+1]) belong to bucket b).
struct ScanHost {
    std::vector<ScanSlot> slots;
    std::vector<int32_t> lev;
    std::vector<float> w;
    std::vector<int> bucket_first;
};

// Device copies of the tables inside a scan workspace.
struct ScanDev {
    ScanSlot *slots;
    int32_t *lev;
    float *w;
    double *betas, *gammas;
    unsigned int *counters;  // one per bucket
};

int scan_num_buckets();
int scan_host_tables(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists,
                     int hist_stride, const int32_t *target_host, const int32_t *pmax_host, int pmax_all,
                     ScanHost *out);
ScanDev scan_dev_tables(void *ws, int num_inst, int hist_stride, int nb, int ng, int per_inst);
// Launch shape of one bucket: the caller's tile, else the cached or timed choice.
int scan_choose_tile(int bucket, const DeviceInfo &dev, const ScanArgs &a, unsigned int *counter,
                     const int32_t *tile, hipStream_t st, TileChoice *out);
// Zeroes the bucket's queue counter with a kernel (no memset node when
// captured) and launches the persistent scan kernel of the bucket.
int scan_launch_bucket(int bucket, const TileChoice &tc, const DeviceInfo &dev, ScanArgs a, unsigned int *counter,
                       hipStream_t st);

// ---- statevector work items ---------------------------------------------------------------
constexpr int kItemMaxP = 16;

struct SvItem {
    int32_t inst;  // caller's instance index
    int32_t out;   // caller's item index (output row)
    double beta, gamma;
};

struct SvItemsArgs {
    const SvItem *items;
    int num_items;
    int n;
    const uint8_t *costs;
    const uint64_t *cost_off;  // per instance
    const int32_t *m;          // per instance
    const int32_t *target;     // per instance
    int num_p;
    int p_list[kItemMaxP];
    float *psol;    // [items][num_p]
    float *energy;  // [items][num_p] or null
};

// Items in launch order (grouped by their instance's n, stable), and the
// groups [first[g], first[g+1]) that share one n, hence one launch.
struct ItemOrder {
    std::vector<int> order;   // launch position -> caller's item index
    std::vector<int> first;   // group boundaries, first.back() == num_items
};

int sv_items_order(const int32_t *n_host, int num_items, const int32_t *item_inst, const DeviceInfo &dev,
                   ItemOrder *out);
// Launches one group: a.items points at the group's first item, a.n is the
// group's n.
int sv_items_launch(const SvItemsArgs &a, const DeviceInfo &dev, hipStream_t st);

}  // namespace gqaoa
