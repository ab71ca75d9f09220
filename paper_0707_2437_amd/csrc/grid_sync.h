// grid_sync.h -- grid-wide synchronisation of the persistent batched
// kernels (batch.hip, step2.hip): the membership of a launch's workgroups,
// a bounded grid barrier between steps, and the per-XCD work counters.
#pragma once

#include <hip/hip_runtime.h>

#include "host.h"
#include "internal.h"

namespace lbm {

// Barrier state of the persistent kernel, in device memory (kBarWords
// 32-bit words, all but the error flag zeroed before every launch):
//   bar[0] arrivals at the current grid barrier, bar[1] its generation,
//   bar[2] error flag (a bounded wait timed out; kept until the host reads it),
//   bar[3] the number of member workgroups, fixed when membership closes,
//   bar[4..5] the membership word (64-bit): bit 63 closed, bits 32..62
//   workgroups joined, bits 0..31 joined workgroups that have arrived at the
//   closing barrier.
constexpr int kBarWords = kPoolBarWords;
constexpr int kBarCtr = 8;  // bar[8..23]: the per-XCD item counters of two consecutive steps
constexpr unsigned long long kClosed = 1ull << 63;

__device__ __forceinline__ unsigned long long* member_word(unsigned* bar)
{
    return reinterpret_cast<unsigned long long*>(bar + 4);
}

// Wait (thread 0) until the generation word moves past gen, for at most
// wait_ticks of the constant-rate device clock; on timeout raise the error
// flag and return false.
__device__ __forceinline__ bool wait_generation(unsigned* bar, unsigned gen, unsigned long long wait_ticks)
{
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (wall_clock64() - t0 > wait_ticks) {
            atomicExch(&bar[2], 1u);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Membership: the workgroups that take part in the launch's grid barriers
// are those that have started when membership closes, so the kernel does
// not depend on every workgroup of the grid being resident at once (the
// occupancy the runtime reports for a launch can exceed what the hardware
// holds, e.g. when scalar registers are the limit). Each workgroup joins
// with one atomic add on the membership word unless it is closed, and
// waits until the whole grid has joined or `grace_ticks` have passed since
// its own join (the resident workgroups start within microseconds of each
// other; without the wait, the first to arrive could close membership
// before the others have joined, which is correct but leaves them idle).
// Joined workgroups then meet at a first barrier, and the arrival that
// completes it (all joined have arrived) closes membership with a
// compare-and-swap that fails if anyone joined meanwhile, so no workgroup
// can join after the count is fixed. A workgroup that starts after closing
// (it was not resident) takes no part and ends. Returns the member count (0: not a member, or a bounded wait
// timed out) and the workgroup's rank in joining order.
__device__ __forceinline__ int join_members(unsigned* bar, unsigned long long wait_ticks,
                                            unsigned long long grace_ticks, int* rank)
{
    __shared__ int sh_count, sh_rank;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long* m = member_word(bar);
        sh_count = 0;
        // join: one fetch-and-add of the joined count; a workgroup that
        // finds membership closed is not a member (its increment after the
        // close is never read)
        unsigned long long old = __hip_atomic_fetch_add(m, 1ull << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!(old & kClosed)) {
            sh_rank = (int)((old >> 32) & 0x7fffffffu);
            const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long t0 = wall_clock64();
            old = __hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (((old >> 32) & 0x7fffffffu) < gridDim.x && wall_clock64() - t0 < grace_ticks) {
                __builtin_amdgcn_s_sleep(2);
                old = __hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // arrive: one fetch-and-add of the arrived count. The arrival that
            // finds every joined workgroup arrived tries once to close with a
            // compare-and-swap from the value it produced; if the word has
            // changed since, a workgroup joined meanwhile, and its own arrival
            // will find the counts equal and close.
            old = __hip_atomic_fetch_add(m, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long now = old + 1ull;
            bool closed = false;
            if ((unsigned)(now & 0xffffffffu) == (unsigned)((now >> 32) & 0x7fffffffu)) {
                unsigned long long expect = now;
                closed = __hip_atomic_compare_exchange_strong(m, &expect, now | kClosed, __ATOMIC_RELAXED,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            bool ok = true;
            if (closed) {
                __hip_atomic_store(&bar[3], (unsigned)((now >> 32) & 0x7fffffffu), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = wait_generation(bar, gen, wait_ticks);
            }
            if (ok) {
                __threadfence();
                sh_count = (int)__hip_atomic_load(&bar[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __syncthreads();
    *rank = sh_rank;
    return sh_count;
}

// Grid barrier among the nblocks members: the last to arrive resets the
// counter (bar[0]) and bumps the generation (bar[1]); the others poll the
// generation with relaxed atomic loads and acquire once it has moved. The
// wait is bounded (wait_generation): on a timeout the workgroup returns
// false, and the kernel then ends in every workgroup (no workgroup can wait
// forever). Only thread 0 of a workgroup touches the barrier words, with
// vector-memory atomics.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, unsigned long long wait_ticks,
                                             unsigned* zero_words = nullptr, int nzero = 0)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();  // this workgroup's stores before its arrival
        const unsigned arrived = atomicAdd(&bar[0], 1u);
        if (arrived == nblocks - 1) {
            atomicExch(&bar[0], 0u);
            for (int k = 0; k < nzero; ++k) atomicExch(&zero_words[k], 0u);  // before the release
            __threadfence();
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else if (!wait_generation(bar, gen, wait_ticks)) {
            ok = 0;
        }
        __threadfence();  // the other workgroups' stores of this step, before the next step's loads
        if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    }
    __syncthreads();
    return ok != 0;
}

// Read a descriptor (or a field of one) through the constant address space.
// The descriptors do not change during a launch; read this way the loads are
// scalar loads, counted apart from the vector loads and stores of the tiles.
// Read as ordinary global memory after the kernel's first stores, the
// compiler would issue them as vector loads (it cannot prove the stores do
// not clobber them), and waiting for them would wait for every store before.
#define LBM_CONST __attribute__((address_space(4)))
template <class V> __device__ __forceinline__ V ldc(const V* p)
{
    V r;
    __builtin_memcpy(&r, (const LBM_CONST V*)p, sizeof(V));
    return r;
}

// Whether a barrier of an earlier launch timed out and the host has not yet
// read the flag (then a launch does nothing). Read once per workgroup, so
// that all its waves take the same branch.
__device__ __forceinline__ bool stale_barrier_error(const unsigned* bar)
{
    __shared__ int flag;
    if (threadIdx.x == 0)
        flag = __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    __syncthreads();
    return flag != 0;
}

// The k-th item of part `part` of a step's items, dealt to nparts parts in
// chunks of ch consecutive items (chunk c to part c mod nparts). With one
// part per XCD, as in the grouped launches, horizontally adjacent tiles,
// which share the cache lines at their common edge, are stepped by the same
// XCD.
__device__ __forceinline__ int part_item(int k, int part, int nparts, int ch)
{
    return ((k / ch) * nparts + part) * ch + k % ch;
}

}  // namespace lbm
