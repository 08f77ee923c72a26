// How many workgroups of a kernel the current device holds at once.  A
// persistent launch (a grid that loops over tiles) is sized by it: with a
// grid larger than the resident count, the workgroups past it start only
// after others have finished all their tiles, and a grid that is not a whole
// multiple of it leaves a second, partly empty generation.
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"

namespace sv {

long long resident_grid(const void *fn, size_t dyn_lds, long long want) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, size_t>, long long> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return want;
    long long g = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find({dev, fn, dyn_lds});
        if (it != cache.end()) {
            g = it->second;
        } else {
            int cus = 0, per = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
                cus = 256;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, dyn_lds) != hipSuccess || per <= 0)
                per = 1;
            g = (long long)cus * per;
            cache[{dev, fn, dyn_lds}] = g;
        }
    }
    return want < g ? want : g;
}

}  // namespace sv
