// batch.hip -- batched forms of the variable-speed-of-sound D2Q9 step
// (Buick & Cosgrove, Sec. 3 Eq. 5): many independent lattices of uneven
// size, tau and c^2 stepped by one launch per step (grouped), or by one
// persistent cooperative launch for many steps with a grid barrier between
// steps. Every tile is processed by vstack_tile (step.h), the same code as
// the single-lattice vertical-stack kernel, so each lattice's result is
// bitwise identical to stepping it alone.
#include <hip/hip_runtime.h>

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

// Grid barrier for the persistent kernel: a counter and a generation word in
// device memory (bar[0], bar[1]; zero at first use; bar[2] is an error flag).
// The last workgroup to arrive resets the counter and bumps the generation;
// the others wait for the bump. The wait is bounded: after `spin_limit`
// polls a workgroup gives up, raises the error flag and returns false, and
// the kernel then ends in every workgroup (no workgroup can wait forever).
// All accesses are vector-memory atomics.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, unsigned spin_limit)
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
            __threadfence();
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (++spins > spin_limit) {
                    atomicExch(&bar[2], 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
        }
        __threadfence();
    }
    __syncthreads();
    if (__hip_atomic_load(&bar[2], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    __syncthreads();
    return ok != 0;
}

// nsteps_max steps of the whole batch in one cooperative launch: every
// workgroup strides over the tiles of a step, then all wait at the grid
// barrier before the next step reads what this one wrote. Launched only
// with a grid that is co-resident (hipLaunchCooperativeKernel checks it).
template <class T, bool SHIFT, int VX, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) void batch_persistent_kernel(const BatchLat* __restrict__ lats,
                                                                   const int* __restrict__ item_lat, int nitems,
                                                                   int nsteps_max, unsigned* bar, unsigned spin_limit)
{
    using C = typename CompT<T>::type;
    __shared__ C lds[NW][64 * VX];
    for (int s = 0; s < nsteps_max; ++s) {
        for (int i = blockIdx.x; i < nitems; i += gridDim.x)
            if (batch_item<T, SHIFT, VX, NW, NTS>(lats, item_lat, i, s, lds)) __syncthreads();
        if (!grid_barrier(bar, gridDim.x, spin_limit)) return;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers.

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
    auto kern = batch_persistent_kernel<T, SHIFT, VX, NW, NTS>;
    int dev = 0, per_cu = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * NW, 0);
    if (e != hipSuccess) return e;
    int grid = per_cu * ncu;
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    if (grid > nitems) grid = nitems;
    if (grid < 1) return hipErrorInvalidConfiguration;
    unsigned spin_limit = 1u << 24;  // ~1 s of polling at one poll per ~64 ns
    void* args[] = {(void*)&lats, (void*)&item_lat, (void*)&nitems, (void*)&s_or_n, (void*)&bar, (void*)&spin_limit};
    return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(64 * NW), args, 0, st);
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
// Persistent: s_or_n steps in one cooperative launch, at most max_grid
// workgroups (<= 0: as many as are co-resident), barrier state in `bar`
// (3 words, zero-initialised; bar[2] becomes 1 if a barrier timed out).
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
