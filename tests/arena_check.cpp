// Host-logic check of the pool's range allocator (arena.h), built with g++
// by test_host_logic.py. The chunks come from a fake allocator that hands
// out aligned addresses without memory behind them (the arena only does
// arithmetic on them) and records what it hands out and gets back.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "arena.h"

namespace {

int fails = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);       \
            ++fails;                                               \
        }                                                          \
    } while (0)

struct Fake {
    using Err = int;
    static constexpr int kOk = 0;
    static inline size_t next = size_t(1) << 40;
    static inline int gets = 0, puts = 0, fail = 0;
    static inline std::set<char*> live;
    static int get(void** p, size_t n)
    {
        if (fail) return 2;
        *p = reinterpret_cast<void*>(next);
        live.insert(static_cast<char*>(*p));
        next += (n + (size_t(1) << 30) - 1) / (size_t(1) << 30) * (size_t(1) << 30) + (size_t(1) << 30);
        ++gets;
        return 0;
    }
    static void put(void* p)
    {
        CHECK(live.erase(static_cast<char*>(p)) == 1);
        ++puts;
    }
};

using A = lbm::Arena<Fake>;
constexpr size_t U = A::kAlign;

}  // namespace

int main()
{
    int err = -1;
    A a;
    // budget of 16 units: the first chunk is exactly the budget (rounded)
    char* r0 = static_cast<char*>(a.take(1, 16 * U - 100, &err));
    CHECK(err == 0 && r0 && a.chunks.size() == 1 && a.chunks[0].size == 16 * U && a.total == 16 * U);
    char* base = a.chunks[0].base;
    CHECK(r0 == base);
    char* r1 = static_cast<char*>(a.take(2 * U, 16 * U, &err));  // [1, 3)
    char* r2 = static_cast<char*>(a.take(U + 1, 16 * U, &err));  // rounded to 2 units: [3, 5)
    CHECK(r1 == base + U && r2 == base + 3 * U);
    CHECK(a.chunks[0].free.size() == 1 && a.chunks[0].free.at(5 * U) == 11 * U);

    // first fit: a freed range is reused before the tail
    a.give(r1, 2 * U);
    char* r3 = static_cast<char*>(a.take(U, 16 * U, &err));
    CHECK(r3 == base + U);  // the front of the freed [1, 3)
    CHECK(a.chunks[0].free.at(2 * U) == U);

    // merging: give back [0,1) and [1,2) around the free [2,3) -> one range [0,3)
    a.give(r0, 1);
    a.give(r3, U);
    CHECK(a.chunks[0].free.size() == 2 && a.chunks[0].free.at(0) == 3 * U && a.chunks[0].free.at(5 * U) == 11 * U);
    // and with the range after: give back [3,5) -> everything free again
    a.give(r2, 2 * U);
    CHECK(a.chunks[0].free.size() == 1 && a.chunks[0].free.at(0) == 16 * U);

    // fill the chunk, then a request beyond the budget gets a chunk of exactly its size
    char* big = static_cast<char*>(a.take(16 * U, 16 * U, &err));
    CHECK(big == base && a.chunks[0].free.empty());
    char* over = static_cast<char*>(a.take(3 * U, 16 * U, &err));
    CHECK(err == 0 && over && a.chunks.size() == 2 && a.chunks[1].size == 3 * U && a.chunks[1].free.empty());

    // a larger budget: new chunks are min(kChunk, what the budget still allows)
    A b;
    char* s0 = static_cast<char*>(b.take(U, 3 * A::kChunk + 5 * U, &err));
    CHECK(s0 && b.chunks.size() == 1 && b.chunks[0].size == A::kChunk);
    char* s1 = static_cast<char*>(b.take(A::kChunk, 3 * A::kChunk + 5 * U, &err));
    CHECK(s1 && b.chunks.size() == 2 && b.chunks[1].size == A::kChunk);
    char* s2 = static_cast<char*>(b.take(A::kChunk, 3 * A::kChunk + 5 * U, &err));
    CHECK(s2 && b.chunks.size() == 3 && b.chunks[2].size == A::kChunk);
    char* s3 = static_cast<char*>(b.take(U, 3 * A::kChunk + 5 * U, &err));  // fits the first chunk's tail
    CHECK(s3 == b.chunks[0].base + U && b.chunks.size() == 3);
    // a range larger than kChunk gets its own chunk
    char* s4 = static_cast<char*>(b.take(A::kChunk + U, 3 * A::kChunk + 5 * U, &err));
    CHECK(s4 && b.chunks.size() == 4 && b.chunks[3].size == A::kChunk + U);

    // a failed chunk allocation reports the allocator's status and changes nothing
    Fake::fail = 1;
    const size_t before = b.total;
    void* none = b.take(4 * A::kChunk, 0, &err);
    CHECK(none == nullptr && err == 2 && b.total == before && b.chunks.size() == 4);
    Fake::fail = 0;

    // every range is a multiple of kAlign from its chunk's base
    for (char* p : {r0, r1, r2, r3, big, over, s0, s1, s2, s3, s4}) {
        bool inside = false;
        for (auto* ar : {&a, &b})
            for (auto& c : ar->chunks)
                if (p >= c.base && p < c.base + c.size) inside = ((p - c.base) % U) == 0;
        CHECK(inside);
    }

    a.release();
    b.release();
    CHECK(a.chunks.empty() && a.total == 0 && b.chunks.empty());
    CHECK(Fake::gets == 6 && Fake::puts == 6 && Fake::live.empty());
    if (fails == 0) std::printf("arena ok\n");
    return fails == 0 ? 0 : 1;
}
