// arena.h -- the range allocator behind a pool's slot memory: ranges of a
// few large allocations (chunks), so that a pool of many small lattices lies
// in a handful of large mappings whatever the process has allocated and
// freed before, and admitting or retiring a lattice allocates and frees
// nothing once the chunks exist. Ranges are multiples of kAlign, taken
// first-fit and merged with free neighbours when given back; a chunk is at
// most kChunk bytes unless one range needs more, and chunks stop growing by
// kChunk once they cover the budget (then a chunk is exactly what the range
// needs). Chunks are freed by release().
//
// Alloc supplies the chunks: Alloc::Err (its status type), Alloc::kOk,
// Err Alloc::get(void** p, size_t n) and void Alloc::put(void* p). The pool
// uses device memory; the host-logic tests use malloc.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace lbm {

template <class Alloc> struct Arena {
    using Err = typename Alloc::Err;
    static constexpr size_t kAlign = size_t(64) << 10;
    static constexpr size_t kChunk = size_t(2) << 30;
    struct Chunk {
        char* base = nullptr;
        size_t size = 0;
        std::map<size_t, size_t> free;  // offset -> length of each free range
    };
    std::vector<Chunk> chunks;
    size_t total = 0;  // bytes of all chunks

    static size_t round(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    // A range of at least n bytes (n rounded up to kAlign), or nullptr with
    // *err set to what Alloc::get returned.
    void* take(size_t n, size_t budget, Err* err)
    {
        *err = Alloc::kOk;
        n = round(n);
        for (auto& c : chunks)
            for (auto it = c.free.begin(); it != c.free.end(); ++it)
                if (it->second >= n) {
                    const size_t off = it->first, len = it->second;
                    c.free.erase(it);
                    if (len > n) c.free[off + n] = len - n;
                    return c.base + off;
                }
        const size_t room = round(budget) > total ? round(budget) - total : 0;
        const size_t size = std::max(n, std::min(kChunk, room));
        Chunk c;
        void* p = nullptr;
        *err = Alloc::get(&p, size);
        if (*err != Alloc::kOk) return nullptr;
        c.base = static_cast<char*>(p);
        c.size = size;
        if (size > n) c.free[n] = size - n;
        chunks.push_back(std::move(c));
        total += size;
        return chunks.back().base;
    }

    // Give back a range that take(n, ...) returned.
    void give(void* p, size_t n)
    {
        n = round(n);
        for (auto& c : chunks) {
            if (static_cast<char*>(p) < c.base || static_cast<char*>(p) >= c.base + c.size) continue;
            size_t off = static_cast<size_t>(static_cast<char*>(p) - c.base);
            auto next = c.free.lower_bound(off);
            if (next != c.free.end() && next->first == off + n) {  // merge with the range after
                n += next->second;
                next = c.free.erase(next);
            }
            if (next != c.free.begin()) {  // merge with the range before
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) {
                    off = prev->first;
                    n += prev->second;
                    c.free.erase(prev);
                }
            }
            c.free[off] = n;
            return;
        }
    }

    void release()
    {
        for (auto& c : chunks)
            if (c.base) Alloc::put(c.base);
        chunks.clear();
        total = 0;
    }
};

}  // namespace lbm
