// Chunk plans of the X-QAOA passes: which tile bits sit in registers at each
// step of a group's mixers. Plain constexpr code, shared by the kernels (as
// template arguments), the host launcher and a host-only test.
#pragma once

#include <cstdint>

namespace gqaoa {

constexpr int kXMaxChunks = 6;

// The register chunks of one group's mixers: chunk k holds tile bits
// [rb[k], rb[k] + R) in registers and applies the qubits of mask[k].
struct XPlan {
    int nchunks;
    int rb[kXMaxChunks];
    int mask[kXMaxChunks];
};

// The chunks for the group on tile bits [mlo, TB): from the top register
// position down by R at a time, never below mlo, each taking the group's bits
// it covers that no earlier chunk took.
constexpr XPlan x_plan(int TB, int R, int mlo) {
    XPlan pl{};
    uint32_t done = 0;
    const uint32_t want = ((1u << TB) - 1u) & ~((1u << mlo) - 1u);
    int rb = TB - R;
    for (;;) {
        int m = 0;
        for (int r = 0; r < R; ++r) {
            const int bit = rb + r;
            if (bit >= mlo && bit < TB && !((done >> bit) & 1u)) {
                m |= 1 << r;
                done |= 1u << bit;
            }
        }
        pl.rb[pl.nchunks] = rb;
        pl.mask[pl.nchunks] = m;
        ++pl.nchunks;
        if (done == want) break;
        rb = rb - R > mlo ? rb - R : mlo;
    }
    return pl;
}

// Group 0 in a pass that only mixes: the loaded layout's chunk first, then
// from tile bit 0 upwards, so that the last chunk is the highest one below it
// and the tile can be stored from there (lanes over runs of >= 128 bytes)
// without an exchange back.
constexpr XPlan x_plan_mix0(int TB, int R) {
    XPlan pl{};
    const int rb0 = TB - R;
    pl.rb[0] = rb0;
    pl.mask[0] = (1 << R) - 1;
    pl.nchunks = 1;
    uint32_t done = ((1u << R) - 1u) << rb0;
    for (int lo = 0; done != (1u << TB) - 1u; lo += R) {
        const int rb = lo + R <= rb0 ? lo : rb0 - R;
        int m = 0;
        for (int r = 0; r < R; ++r)
            if (!((done >> (rb + r)) & 1u)) {
                m |= 1 << r;
                done |= 1u << (rb + r);
            }
        pl.rb[pl.nchunks] = rb;
        pl.mask[pl.nchunks] = m;
        ++pl.nchunks;
    }
    return pl;
}
// The compile-time plans: MLO >= 0 a group on tile bits [MLO, TB); kXPlanMix0
// group 0's plan for a mixing-only pass.
constexpr int kXPlanMix0 = 64;
constexpr XPlan x_plan_id(int TB, int R, int id) { return id == kXPlanMix0 ? x_plan_mix0(TB, R) : x_plan(TB, R, id); }

}  // namespace gqaoa
