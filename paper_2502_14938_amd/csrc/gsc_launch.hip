// Launch shapes of the grid-stride kernels.
#include <mutex>
#include <unordered_map>

#include "gsc_common.h"

namespace gsc {

int resident_blocks(const void* kernel, int threads) {
    static std::mutex mu;
    static std::unordered_map<uint64_t, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const uint64_t key = (uint64_t)(uintptr_t)kernel ^ ((uint64_t)dev << 56) ^ ((uint64_t)threads << 40);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    const int g = per_cu * cus;
    cache.emplace(key, g);
    return g;
}

}  // namespace gsc
