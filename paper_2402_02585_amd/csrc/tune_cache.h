// Launch shapes of the batched scan and the text file that persists the
// autotuner's choices. Host code only (no HIP types), so a plain C++ compiler
// can build it for tests of the parser.
#pragma once

#include <cstdio>
#include <map>
#include <string>

namespace gqaoa {

struct TileChoice {
    int waves, blocks_per_cu;
};

// Launch shapes the scan kernels accept: 1, 2 or 4 waves per block (the
// kernels are compiled for at most 4 waves and size their LDS for 4) and
// 1..32 blocks per compute unit.
inline bool tile_valid(int waves, int blocks_per_cu) {
    return (waves == 1 || waves == 2 || waves == 4) && blocks_per_cu >= 1 && blocks_per_cu <= 32;
}

// Reads "key waves blocks_per_cu" lines into `out` until the first line that
// does not parse; entries with a shape tile_valid rejects are skipped (the
// bucket is then timed again). Returns the number of entries skipped.
inline int tune_cache_read(FILE *f, std::map<std::string, TileChoice> &out) {
    char key[256];
    int wv = 0, bpc = 0, skipped = 0;
    while (std::fscanf(f, "%255s %d %d", key, &wv, &bpc) == 3) {
        if (tile_valid(wv, bpc))
            out[key] = TileChoice{wv, bpc};
        else
            ++skipped;
    }
    return skipped;
}

inline void tune_cache_write(FILE *f, const std::map<std::string, TileChoice> &in) {
    for (const auto &kv : in) std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.waves, kv.second.blocks_per_cu);
}

}  // namespace gqaoa
