// First-fit allocator over a range of 8-byte words (the serving result
// arena): free runs kept by offset, neighbours merged on release.  Host-only
// (no device calls), so its policy is checked on the CPU.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace lap {

class WordArena {
   public:
    explicit WordArena(int64_t words = 0) { reset(words); }

    void reset(int64_t words) {
        runs_.clear();
        size_ = words;
        if (words > 0) runs_[0] = words;
    }

    // the lowest-offset free run that holds `words` words, or -1
    int64_t alloc(int64_t words) {
        if (words <= 0) return -1;
        for (auto it = runs_.begin(); it != runs_.end(); ++it) {
            if (it->second >= words) {
                const int64_t off = it->first, len = it->second;
                runs_.erase(it);
                if (len > words) runs_[off + words] = len - words;
                return off;
            }
        }
        return -1;
    }

    // give back [off, off + words); returns false (and changes nothing) if
    // the range is outside the arena or overlaps a free run
    bool release(int64_t off, int64_t words) {
        if (words <= 0 || off < 0 || off + words > size_) return false;
        auto nx = runs_.lower_bound(off);
        if (nx != runs_.end() && nx->first < off + words) return false;
        if (nx != runs_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second > off) return false;
        }
        auto it = runs_.emplace(off, words).first;
        nx = std::next(it);
        if (nx != runs_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            runs_.erase(nx);
        }
        if (it != runs_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                runs_.erase(it);
            }
        }
        return true;
    }

    int64_t size() const { return size_; }
    int64_t free_words() const {
        int64_t f = 0;
        for (const auto &r : runs_) f += r.second;
        return f;
    }
    int64_t runs() const { return (int64_t)runs_.size(); }

   private:
    std::map<int64_t, int64_t> runs_;   // offset -> length of each free run
    int64_t size_ = 0;
};

}  // namespace lap
