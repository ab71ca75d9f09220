// batch.hip -- batched forms of the variable-speed-of-sound D2Q9 step
// (Buick & Cosgrove, Sec. 3 Eq. 5): many independent lattices of uneven
// size, tau and c^2 stepped by one launch per step (grouped), or by one
// persistent launch for many steps with a grid barrier between
// steps. Every tile is processed by vstack_tile (step.h), the same code as
// the single-lattice vertical-stack kernel, so each lattice's result is
// bitwise identical to stepping it alone.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "grid_sync.h"
#include "host.h"
#include "internal.h"
#include "step.h"

namespace lbm {

// One work item: up to per_item consecutive tiles (row-band order: adjacent
// strips of one row group, then the next group) of one lattice. The item's
// lattice comes from a direct map, so a workgroup pays two dependent loads
// (map, descriptor) per item instead of a search per tile. Returns whether
// the item had work (uniform per workgroup); the caller places a barrier
// before reusing lds.
template <class T, bool SHIFT, int VX, int NW, bool NTS>
__device__ __forceinline__ bool batch_item(const BatchLat* __restrict__ lats, const int* __restrict__ item_lat, int i,
                                           int s, typename CompT<T>::type (&lds)[NW][64 * VX])
{
    const BatchLat& L = lats[item_lat[i]];
    if (s >= L.nsteps) return false;
    const bool odd = ((L.t0 + s) & 1) != 0;
    const void* src = odd ? L.tile.dst : L.tile.src;
    void* dst = odd ? const_cast<void*>(L.tile.src) : L.tile.dst;
    const int t0 = (i - L.item_begin) * L.per_item;
    const int t1 = min(t0 + L.per_item, L.ntiles);
    for (int t = t0; t < t1; ++t) {
        if (t > t0) __syncthreads();  // lds of the previous tile is still being read
        // pools step the paper's model: centred on the weights (see Centre)
        vstack_tile<T, SHIFT, VX, NW, NTS, false, false>(L.tile, src, dst, t % L.tile.nstrips, t / L.tile.nstrips,
                                                         lds);
    }
    return true;
}

// One step s of every lattice of the batch; one workgroup per item, items
// of a lattice contiguous, dealt to the XCDs in chunks of ch items
// (xcd_tile; the grid is a multiple of 8 ch, or of 8 for ch <= 0).
template <class T, bool SHIFT, int VX, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) void batch_step_kernel(const BatchLat* __restrict__ lats,
                                                             const int* __restrict__ item_lat, int nitems, int s,
                                                             int ch)
{
    using C = typename CompT<T>::type;
    __shared__ C lds[NW][64 * VX];
    const int i = xcd_tile(blockIdx.x, gridDim.x, ch);
    if (i >= nitems) return;
    batch_item<T, SHIFT, VX, NW, NTS>(lats, item_lat, i, s, lds);
}

// A workgroup's place in a step of the persistent kernel: tile t of work
// item i, which belongs to lattice L; t1 ends the item's tiles. L == nullptr:
// the workgroup has no more work in this step.
struct Unit {
    const BatchLat* L;
    int i, t, t1;
};

// The first of items i, i + G, i + 2 G, ... whose lattice takes step s.
__device__ __forceinline__ Unit find_unit(const BatchLat* __restrict__ lats, const int* __restrict__ item_lat,
                                          int nitems, int i, int G, int s)
{
    for (; i < nitems; i += G) {
        const BatchLat* L = &lats[ldc(&item_lat[i])];
        if (s < ldc(&L->nsteps)) {
            const int per = ldc(&L->per_item);
            const int t0 = (i - ldc(&L->item_begin)) * per;
            return Unit{L, i, t0, min(t0 + per, ldc(&L->ntiles))};
        }
    }
    return Unit{nullptr, i, 0, 0};
}

// nsteps_max steps of the whole batch in one launch whose G member
// workgroups (join_members; all of the grid when it is resident at once)
// meet at a grid barrier between steps.
// Work is taken dynamically: the items are split into parts, one per XCD
// when the whole grid joined and is a multiple of 8 workgroups (workgroup b
// runs on XCD b mod 8), else a single part; each part has a counter per
// step (two steps' sets alternate; the barrier's last arriver zeroes the
// set of the next step), and a member takes its part's next item
// (part_item) with one atomic add, issued with the window loads of its
// current item's last tile, so the wait for those loads also covers it.
// Members that finish early take more items, so a step ends when the work
// does, whatever the speed of each workgroup. Each tile is processed as in
// the grouped kernel (issue, land, barrier, relax); the LDS holding the
// densities is double-buffered, so consecutive tiles need one workgroup
// barrier each. All members meet at the grid barrier between steps, since
// step s + 1 reads what step s wrote.
template <class T, bool SHIFT, int VX, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(sizeof(T) <= 4 && VX <= 2 ? 8 : 1, 8))) void batch_persistent_kernel(const BatchLat* __restrict__ lats,
                                                                   const int* __restrict__ item_lat, int nitems,
                                                                   int nsteps_max, int ch, unsigned* bar,
                                                                   unsigned long long wait_ticks,
                                                                   unsigned long long grace_ticks)
{
    using C = typename CompT<T>::type;
    using V = VTile<T, SHIFT, VX, NW, NTS, false, false>;  // pools step the paper's model, centred on the weights
    __shared__ C lds[2][NW][64 * VX];
    __shared__ int next_item[2];
    if (stale_barrier_error(bar)) return;
    int rank = 0;
    const int G = join_members(bar, wait_ticks, grace_ticks, &rank);
    if (G == 0) return;
    const bool by_xcd = G == (int)gridDim.x && G % 8 == 0;
    const int nparts = by_xcd ? 8 : 1;
    const int part = by_xcd ? (int)(blockIdx.x & 7u) : 0;
    const int chunk = ch > 0 ? ch : 1;
    int buf = 0;
    for (int s = 0; s < nsteps_max; ++s) {
        unsigned* ctr = bar + kBarCtr + (s & 1) * 8 + part;
        // the item of counter value k (nitems: none left)
        auto take = [&](unsigned k) { return min(part_item((int)k, part, nparts, chunk), nitems); };
        if (threadIdx.x == 0) next_item[buf] = take(atomicAdd(ctr, 1u));
        __syncthreads();
        int i = next_item[buf];
        buf ^= 1;  // the slot just read is not written again before the next barrier
        while (i < nitems) {
            const BatchLat* L = &lats[ldc(&item_lat[i])];
            if (s >= ldc(&L->nsteps)) {  // this lattice takes fewer steps: the next item
                if (threadIdx.x == 0) next_item[buf] = take(atomicAdd(ctr, 1u));
                __syncthreads();
                i = next_item[buf];
                buf ^= 1;
                continue;
            }
            StepTile a = ldc(&L->tile);
            if ((ldc(&L->t0) + s) & 1) {
                const void* b = a.src;
                a.src = a.dst;
                a.dst = const_cast<void*>(b);
            }
            const int per = ldc(&L->per_item);
            const int t0 = (i - ldc(&L->item_begin)) * per;
            const int t1 = min(t0 + per, ldc(&L->ntiles));
            for (int t = t0; t < t1; ++t) {
                const bool last = t + 1 == t1;
                const int strip = t % a.nstrips;
                const VRow r = vrow<VX, NW>(a.g, strip, t / a.nstrips);
                unsigned k = 0;
                if (last && threadIdx.x == 0) k = atomicAdd(ctr, 1u);
                // as vstack_tile, with the next item published before the barrier
                auto run = [&](auto edge) {
                    V v;
                    v.af = {};
                    if (r.load) {
                        v.template issue_rows<decltype(edge)::value>(a, a.src, r);
                        v.land_rows(a, r, lds[buf]);
                    }
                    if (last && threadIdx.x == 0) next_item[buf] = take(k);
                    __syncthreads();  // the tile's densities are in lds[buf]
                    v.relax(a, a.dst, r, lds[buf]);
                };
                if constexpr (GhostCols<T>::value) run(std::false_type{});
                else if (edge_strip<T, VX>(a.g, strip)) run(std::true_type{});
                else run(std::false_type{});
                if (last) i = next_item[buf];
                buf ^= 1;
            }
        }
        if (!grid_barrier(bar, G, wait_ticks, bar + kBarCtr + ((s + 1) & 1) * 8, s + 1 < nsteps_max ? 8 : 0)) return;
    }
}

// Zero the barrier state before a persistent launch, all but the error
// flag (bar[2]), which is kept until the host has read it.
__global__ void barrier_reset_kernel(unsigned* bar)
{
    const int w = threadIdx.x;
    if (w < kBarWords && w != 2) bar[w] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers.

hipError_t persistent_setup(const void* kern, int threads, int max_grid, int* ch, int* grid_out,
                            unsigned long long* wait_ticks, unsigned long long* grace_ticks, unsigned* bar,
                            hipStream_t st)
{
    int dev = 0, per_cu = 0, ncu = 0, clock_khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
    if (e != hipSuccess) return e;
    // The grid the runtime reports as resident at once; the workgroups that
    // are not (if the report is high) take no part (join_members).
    int grid = per_cu * ncu;
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    // a grid that is a multiple of 8 ch (or of 8) makes xcd_tile a permutation
    if (*ch > 0 && grid >= 8 * *ch) grid = grid / (8 * *ch) * (8 * *ch);
    else if (grid >= 8) {
        *ch = 0;
        grid = grid / 8 * 8;
    } else {
        *ch = -1;
    }
    if (grid < 1 || clock_khz <= 0) return hipErrorInvalidConfiguration;
    // bound on one workgroup's wait at a grid barrier (LBM_BARRIER_WAIT_US
    // sets it for tests of the timeout path; default 1 s)
    double wait_us = 1e6;
    if (const char* ev = std::getenv("LBM_BARRIER_WAIT_US")) {
        const double v = std::atof(ev);
        if (v >= 0.0 && v <= 1e8) wait_us = v;
    }
    *wait_ticks = (unsigned long long)(wait_us * 1e-3 * clock_khz);
    // how long a workgroup waits for the rest of the grid to join (20 us)
    *grace_ticks = (unsigned long long)(20.0 * 1e-3 * clock_khz);
    *grid_out = grid;
    hipLaunchKernelGGL(barrier_reset_kernel, dim3(1), dim3(64), 0, st, bar);
    return hipGetLastError();
}

template <class T, bool SHIFT, int VX, int NW, bool NTS>
static hipError_t launch_batch_t(bool persistent, const BatchLat* lats, const int* item_lat, int nitems,
                                 int s_or_n, int max_grid, int ch, unsigned* bar, hipStream_t st)
{
    if (!persistent) {
        const int q = ch > 0 ? 8 * ch : 8;
        const int grid = (nitems + q - 1) / q * q;
        if (!grid_fits(grid, 64 * NW)) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL((batch_step_kernel<T, SHIFT, VX, NW, NTS>), dim3(grid), dim3(64 * NW), 0, st, lats,
                           item_lat, nitems, s_or_n, ch);
        return hipGetLastError();
    }
    int grid = 0;
    unsigned long long wait_ticks = 0, grace_ticks = 0;
    hipError_t e = persistent_setup((const void*)batch_persistent_kernel<T, SHIFT, VX, NW, NTS>, 64 * NW, max_grid,
                                    &ch, &grid, &wait_ticks, &grace_ticks, bar, st);
    if (e != hipSuccess) return e;
    const int threads = 64 * NW;
    // An ordinary launch: the membership (join_members) makes the kernel
    // correct whether or not every workgroup is resident at once, so the
    // cooperative-launch guarantee is not needed.
    hipLaunchKernelGGL((batch_persistent_kernel<T, SHIFT, VX, NW, NTS>), dim3(grid), dim3(threads), 0, st, lats,
                       item_lat, nitems, s_or_n, ch, bar, wait_ticks, grace_ticks);
    return hipGetLastError();
}

template <class T, bool SHIFT, int VX>
static hipError_t launch_batch_nw(int nw, bool nts, bool persistent, const BatchLat* lats, const int* item_lat,
                                  int nitems, int s_or_n, int max_grid, int ch, unsigned* bar, hipStream_t st)
{
#define LBM_B(NWV)                                                                                                 \
    return nts ? launch_batch_t<T, SHIFT, VX, NWV, true>(persistent, lats, item_lat, nitems, s_or_n, max_grid, ch, \
                                                         bar, st)                                                    \
               : launch_batch_t<T, SHIFT, VX, NWV, false>(persistent, lats, item_lat, nitems, s_or_n, max_grid, ch, \
                                                          bar, st)
    switch (nw) {
    case 4: LBM_B(4);
    case 8: LBM_B(8);
    case 16: LBM_B(16);
    default: return hipErrorInvalidValue;
    }
#undef LBM_B
}

template <class T, bool SHIFT>
static hipError_t launch_batch_vx(int vx, int nw, bool nts, bool persistent, const BatchLat* lats,
                                  const int* item_lat, int nitems, int s_or_n, int max_grid, int ch, unsigned* bar,
                                  hipStream_t st)
{
#define LBM_BN(VXV) launch_batch_nw<T, SHIFT, VXV>(nw, nts, persistent, lats, item_lat, nitems, s_or_n, max_grid, ch, bar, st)
    switch (vx) {
    case 1: return LBM_BN(1);
    case 2: return LBM_BN(2);
    case 4: return LBM_BN(4);
    default: return hipErrorInvalidValue;
    }
#undef LBM_BN
}

// Grouped (persistent = false): step s_or_n of the batch, one launch, one
// workgroup per item, items dealt to the XCDs in chunks of ch items (<= 0:
// one contiguous run per XCD).
// Persistent: s_or_n steps in one launch, at most max_grid
// workgroups (<= 0: as many as the runtime reports resident), items taken
// dynamically in chunks of ch per XCD, barrier and counter state in `bar`
// (kPoolBarWords words, all but bar[2] reset on the stream before the
// launch; bar[2] becomes 1 if a barrier timed out, and a launch that finds
// it set does nothing).
hipError_t launch_batch(int dtype, int vx, int nw, bool nts, bool persistent, const BatchLat* lats,
                        const int* item_lat, int nitems, int s_or_n, int max_grid, int ch, unsigned* bar,
                        hipStream_t st)
{
#define LBM_BV(T, S) launch_batch_vx<T, S>(vx, nw, nts, persistent, lats, item_lat, nitems, s_or_n, max_grid, ch, bar, st)
    switch (dtype) {
    case 0: return LBM_BV(double, false);
    case 1: return LBM_BV(float, false);
    case 2: return LBM_BV(float, true);
    case 3: return LBM_BV(_Float16, true);
    default: return hipErrorInvalidValue;
    }
#undef LBM_BV
}

}  // namespace lbm
