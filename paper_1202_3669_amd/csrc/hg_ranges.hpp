// hg_ranges.hpp -- first-fit allocation of ranges of [0, size), with
// returned ranges coalesced: the carving of the serving loop's staging
// region and of a context's device and pinned pools (one region allocated
// once and reused, Sec. 3.1 / 3.2.3).  Not thread-safe; callers lock.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace hg {

class Ranges {
  public:
    void init(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool fits(uint64_t n) const {
        for (const auto &kv : free_)
            if (kv.second >= n) return true;
        return false;
    }
    bool take(uint64_t n, uint64_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void give(uint64_t off, uint64_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

}  // namespace hg
