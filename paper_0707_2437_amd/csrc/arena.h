// arena.h -- the range allocator behind a pool's slot memory: ranges of a
// few large allocations (chunks), so that a pool of many small lattices lies
// in a handful of large mappings whatever the process has allocated and
// freed before, and admitting or retiring a lattice allocates and frees
// nothing once the chunks exist. Ranges are multiples of kAlign, taken
// first-fit and merged with free neighbours when given back. A new chunk is
// kChunk bytes, or what the budget still allows if that is less, or exactly
// the range when the budget is used up. Ranges need not fill their chunks
// (a chunk's tail may be too small for the next range), so the chunks may
// exceed the budget, by at most kChunk: when a new chunk would go past that,
// chunks that are entirely free are given back to the allocator first, and
// if that does not make room take() fails with Alloc::kNoMem and the caller
// waits for ranges to be given back. Chunks are freed by release().
//
// Alloc supplies the chunks: Alloc::Err (its status type), Alloc::kOk,
// Alloc::kNoMem, Err Alloc::get(void** p, size_t n) and void Alloc::put(void*
// p). The pool uses device memory; the host-logic tests use a fake.
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
    // Most the chunks may hold for a budget: the budget plus one chunk of
    // room for ranges that do not pack.
    static size_t limit(size_t budget) { return round(budget) + kChunk; }

    static bool empty(const Chunk& c) { return c.free.size() == 1 && c.free.begin()->second == c.size; }

    // Give back to the allocator every chunk with no range in use.
    void drop_empty()
    {
        for (size_t k = 0; k < chunks.size();) {
            if (empty(chunks[k])) {
                Alloc::put(chunks[k].base);
                total -= chunks[k].size;
                chunks.erase(chunks.begin() + (long)k);
            } else {
                ++k;
            }
        }
    }

    // A range of at least n bytes (n rounded up to kAlign), or nullptr with
    // *err set to Alloc::kNoMem (no room within limit(budget)) or to what
    // Alloc::get returned.
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
        const size_t cap = limit(budget);
        if (total + n > cap) drop_empty();
        if (total + n > cap) {
            *err = Alloc::kNoMem;
            return nullptr;
        }
        const size_t b = round(budget);
        const size_t size = std::max(n, std::min(kChunk, b > total ? b - total : 0));
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
