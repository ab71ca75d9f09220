// Host-logic check of the pool's range allocator (arena.h), built with g++
// by test_host_logic.py. The chunks come from a fake allocator that hands
// out aligned addresses without memory behind them (the arena only does
// arithmetic on them) and records what it hands out and gets back.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

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
    static constexpr int kNoMem = 3;
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

    // fill the chunk; a request beyond the budget gets a chunk of exactly its size
    char* big = static_cast<char*>(a.take(16 * U, 16 * U, &err));
    CHECK(big == base && a.chunks[0].free.empty());
    char* over = static_cast<char*>(a.take(3 * U, 16 * U, &err));
    CHECK(err == 0 && over && a.chunks.size() == 2 && a.chunks[1].size == 3 * U && a.chunks[1].free.empty());
    // ... but not past the budget plus one chunk: that fails and allocates nothing
    char* none0 = static_cast<char*>(a.take(A::kChunk, 16 * U, &err));
    CHECK(none0 == nullptr && err == Fake::kNoMem && a.chunks.size() == 2 && a.total == 19 * U);

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
    char* s4 = static_cast<char*>(b.take(A::kChunk + U, 5 * A::kChunk, &err));
    CHECK(s4 && b.chunks.size() == 4 && b.chunks[3].size == A::kChunk + U);

    // a failed chunk allocation reports the allocator's status and changes nothing
    Fake::fail = 1;
    const size_t before = b.total;
    void* none = b.take(3 * A::kChunk, 8 * A::kChunk, &err);
    CHECK(none == nullptr && err == 2 && b.total == before && b.chunks.size() == 4);
    Fake::fail = 0;

    // no room within the limit: chunks with no range in use are given back first
    A c;
    char* c0 = static_cast<char*>(c.take(4 * U, 10 * U, &err));  // chunk 0: 10 units
    c.give(c0, 4 * U);                                           // chunk 0 now empty
    char* c1 = static_cast<char*>(c.take(A::kChunk + 4 * U, 10 * U, &err));  // > limit - 10 units
    CHECK(c1 && err == 0 && c.chunks.size() == 1 && c.chunks[0].size == A::kChunk + 4 * U);

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
    c.release();
    CHECK(a.chunks.empty() && a.total == 0 && b.chunks.empty() && c.chunks.empty());
    CHECK(Fake::gets == Fake::puts && Fake::live.empty());

    // churn: a served job stream (square FP32 lattices of side 2^U[7, 11],
    // A and B buffers, seeded lifetimes) under a budget that is too small
    // for all of them: the chunks never exceed the budget, ranges in use
    // never overlap, and some requests wait for others to be given back
    {
        A d;
        const size_t budget = size_t(8) << 30;
        unsigned long long s = 0x9e3779b97f4a7c15ULL;
        auto rnd = [&]() {  // SplitMix64
            unsigned long long z = (s += 0x9e3779b97f4a7c15ULL);
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
            return z ^ (z >> 31);
        };
        struct Live { char* p; size_t n; int until; };
        std::vector<Live> live;
        int refused = 0, served = 0;
        for (int t = 0; t < 20000; ++t) {
            for (size_t k = 0; k < live.size();)
                if (live[k].until <= t) {
                    d.give(live[k].p, live[k].n);
                    live[k] = live.back();
                    live.pop_back();
                } else {
                    ++k;
                }
            const double u = (rnd() >> 11) * (1.0 / 9007199254740992.0);
            const size_t side = (size_t)std::pow(2.0, 7.0 + 4.0 * u);
            const size_t n = 2 * 9 * side * side * 4 + (side << 8);
            char* p = static_cast<char*>(d.take(n, budget, &err));
            CHECK(d.total <= A::limit(budget));
            if (!p) {
                CHECK(err == Fake::kNoMem);
                ++refused;
                continue;
            }
            ++served;
            const size_t len = A::round(n);
            for (const Live& l : live) CHECK(p + len <= l.p || l.p + l.n <= p);
            live.push_back({p, len, t + 1 + (int)(rnd() % 400)});
        }
        std::fprintf(stderr, "churn: %d served, %d refused, %zu chunks\n", served, refused, d.chunks.size());
        CHECK(refused > 0 && served > 1000);
        for (const Live& l : live) d.give(l.p, l.n);
        d.drop_empty();
        CHECK(d.chunks.empty() && d.total == 0);
        d.release();
    }

    // a budget that is exactly the sum of the ranges admits all of them,
    // in any order (the chunks' unfilled tails stay within the allowance)
    {
        A e;
        unsigned long long s = 7;
        std::vector<size_t> sizes;
        size_t sum = 0;
        for (int k = 0; k < 256; ++k) {
            s = s * 6364136223846793005ULL + 1442695040888963407ULL;
            const size_t side = 64 + (size_t)((s >> 33) % 961);
            sizes.push_back(A::round(2 * 9 * side * side * 4 + 4096));
            sum += sizes.back();
        }
        int got = 0;
        for (size_t n : sizes) got += e.take(n, sum, &err) != nullptr;
        CHECK(got == 256 && e.total <= A::limit(sum));
        e.release();
    }
    CHECK(Fake::live.empty());
    if (fails == 0) std::printf("arena ok\n");
    return fails == 0 ? 0 : 1;
}
