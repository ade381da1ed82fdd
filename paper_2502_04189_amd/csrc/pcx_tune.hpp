// pcx_tune.hpp -- autotuner of per-size-class launch shapes (x/y tile sizes,
// FFT radix splits, z lanes per line) and its text cache.
#pragma once

#include <map>
#include <string>

#include "pcx_plan.hpp"

namespace pcx {

struct TuneCache {
    std::map<std::string, std::pair<TuneParams, RadixChoice>> m;
    static std::string key(const pcx_grid &g, int prec);
    bool load(const char *path);
    bool save(const char *path) const;
    bool lookup(const pcx_grid &g, int prec, TuneParams &tp, RadixChoice &rc) const;
    void store(const pcx_grid &g, int prec, const TuneParams &tp, const RadixChoice &rc);
};

// Times candidate shapes of each pass on scratch data of this grid and
// returns the fastest per pass.  grouped: time the batch's grouped kernels
// (one-domain item lists), else the single-domain kernels of a plan.
pcx_status autotune_class(const pcx_grid &g, int prec, hipStream_t s, TuneParams &tp, RadixChoice &rc,
                          bool grouped);

} // namespace pcx
