// step2.hip -- two steps of the variable-speed-of-sound D2Q9 step (Buick &
// Cosgrove, Sec. 3 Eq. 5) per pass over memory (temporal blocking).
//
// A single step moves 9 loads and 9 stores per site; the single-step
// kernels (kernels.hip) run close to the HBM bound for that traffic. A
// two-step tile loads its rows once, keeps the first step's results in LDS
// and writes only the second step's, so the bytes per site update fall
// towards half (the tile's halo rows and lanes are loaded but not written).
//
// Tile: strip `strip` (step2_cols(VX) columns) and row group `grp`
// (step2_rows(NW) rows), processed by a workgroup of NW waves. Wave w holds
// row y0 - 3 + w, lane l the VX columns from x0 + (l - HL) VX, with HL =
// step2_halo_lanes(VX) (step2.h). Rows and columns outside the lattice are
// periodic images (Sec. 4), gathered from the wrapped positions. Phases,
// separated by workgroup barriers:
//   1. the waves gather their rows from memory (Eq. 5, left-hand side) and
//      publish the densities of their columns in LDS;
//   2. waves 1 .. NW-2 relax (first step) into LDS, rounded to the storage
//      type: the values a single step would store;
//   3. waves 2 .. NW-3 gather from those and publish the new densities;
//   4. waves 3 .. NW-4, inner lanes only, relax (second step) and write.
// Every site's arithmetic is the single-step code of step.h (VTileF) on the
// same inputs, so a two-step pass gives the bits of two single steps.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "step.h"
#include "step2.h"

namespace lbm {

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Window gather (the columns of window_loads in step.h) for a lane whose
// window may reach past a lattice edge: every element loaded on its own
// from its source column taken mod nx. r is a row in [0, ny).
template <class T, int NV>
__device__ __forceinline__ void gather_wrapped(const char* const (&pb)[9], const Geom& g, int r, int x,
                                               Pack<T, NV> (&v)[9])
{
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr unsigned es = sizeof(T);
    const char* rb[9];
    row_bases<T>(pb, g, r, rb);
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int s = wrap_mod(x + j - 1 - ex[i], g.nx);
            v[i].v[j] = ld_g<T>(rb[i] + (size_t)((unsigned)(s + 2) * es));
        }
}

template <class T, bool SHIFT, int VX, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) void step2_vstack_kernel(StepTile a, int ntiles)
{
    using C = typename CompT<T>::type;
    constexpr bool RC = ModelCentred<C>::value;
    using V = VTileF<T, SHIFT, VX, NW, NTS, false, RC>;
    constexpr int HL = step2_halo_lanes(VX);
    constexpr int W2 = step2_cols(VX);
    constexpr int R2 = step2_rows(NW);
    static_assert(R2 >= 1, "a two-step tile needs at least 7 waves");
    constexpr int LW = 64 * VX + 4;  // an LDS plane row: the lanes' columns and two more on each side
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    __shared__ C rho[NW][64 * VX];   // densities of the lanes' columns, one row per wave
    __shared__ T fs[NW - 2][9][LW];  // first-step results of waves 1 .. NW - 2

    const int t = xcd_tile(blockIdx.x, gridDim.x, a.xcd_chunk);
    if (t >= ntiles) return;
    const Geom g = a.g;
    const int strip = t % a.nstrips, grp = t / a.nstrips;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int y0 = grp * R2;
    const int nrows = min(R2, g.ny - y0);
    const int y = y0 - 3 + wave;
    const int xs = strip * W2;
    const int x = xs + (lane - HL) * VX;
    // The windows of the whole strip (columns x - 2 .. x + VX + 1 of every
    // lane) lie inside the lattice, or some elements wrap.
    const bool edge = xs - HL * VX - 2 < 0 || xs + (64 - HL) * VX + 2 > g.nx;
    const CoefC<C> k = coef_c<C>(a.c);
    const Centre<C> cn = centre_c<C, RC>(a.c);
    const int col = lane * VX + 2;  // LDS column of the lane's first column

    V v;
    v.af = {};
    // 1. Gather from memory; waves past the last row the group needs idle.
    if (wave <= nrows + 5) {
        const char* sb[9];
        src_bases<T>(a.src, g, sb);
        const int yw = wrap_mod(y, g.ny);
        if (edge) gather_wrapped<T, VX + 2>(sb, g, yw, x, v.raw);
        else gather_raw<T, VX + 2, T, VX + 2, false>(sb, g, yw, x, v.raw);
        v.land_regs(a);
#pragma unroll
        for (int j = 0; j < VX; ++j) rho[wave][lane * VX + j] = v.w[j + 1];
    }
    __syncthreads();
    // 2. First step, every lane, into LDS.
    if (wave >= 1 && wave <= min(nrows + 4, NW - 2)) {
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            // undivided central differences at time t (Sec. 4)
            const C gx = v.w[j + 2] - v.w[j];
            const C gy = rho[wave + 1][lane * VX + j] - rho[wave - 1][lane * VX + j];
            C o[9];
            collide<T, SHIFT, C, VX, RC>(v.d, j, v.w[j + 1], gx, gy, k, cn, o);
#pragma unroll
            for (int i = 0; i < 9; ++i) fs[wave - 1][i][col + j] = from_d<T, SHIFT, C>(o[i], i, cn);
        }
    }
    __syncthreads();
    // 3. Second gather, from LDS: f_i at column c of row y is the first
    // step's S_i at column c - e_ix of row y - e_iy. The halo lanes read two
    // LDS columns that nothing wrote; their results are never written.
    const bool act3 = wave >= 2 && wave <= min(nrows + 3, NW - 3);
    if (act3) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < VX + 2; ++j) v.raw[i].v[j] = fs[wave - ey[i] - 1][i][col - 1 + j - ex[i]];
        v.land_regs(a);
#pragma unroll
        for (int j = 0; j < VX; ++j) rho[wave][lane * VX + j] = v.w[j + 1];
    }
    __syncthreads();
    // 4. Second step: the group's rows, inner lanes, columns inside the lattice.
    VRow r;
    r.wave = wave;
    r.lane = lane;
    r.y = y;
    r.x = x;
    r.nv = min(VX, g.nx - x);
    r.load = act3;
    r.relax = wave >= 3 && wave <= nrows + 2 && lane >= HL && lane < 64 - HL && r.nv > 0;
    v.relax_g(a, a.dst, r, [&](int j) { return rho[wave + 1][lane * VX + j] - rho[wave - 1][lane * VX + j]; });
}

template <class T, bool SHIFT, int VX, int NW>
static hipError_t launch2_t(bool nts, const StepTile& t, hipStream_t st)
{
    const int ntiles = t.nstrips * t.nchunks;  // strips x row groups
    const int q = t.xcd_chunk > 0 ? 8 * t.xcd_chunk : 8;
    const int grid = (ntiles + q - 1) / q * q;
    if (!grid_fits(grid, 64 * NW)) return hipErrorInvalidConfiguration;
    const dim3 gd(grid), bd(64 * NW);
    if (nts) hipLaunchKernelGGL((step2_vstack_kernel<T, SHIFT, VX, NW, true>), gd, bd, 0, st, t, ntiles);
    else hipLaunchKernelGGL((step2_vstack_kernel<T, SHIFT, VX, NW, false>), gd, bd, 0, st, t, ntiles);
    return hipGetLastError();
}

template <class T, bool SHIFT, int VX>
static hipError_t launch2_nw(int nw, bool nts, const StepTile& t, hipStream_t st)
{
    switch (nw) {
    case 12: return launch2_t<T, SHIFT, VX, 12>(nts, t, st);
    case 16: return launch2_t<T, SHIFT, VX, 16>(nts, t, st);
    default: return hipErrorInvalidValue;
    }
}

template <class T, bool SHIFT>
static hipError_t launch2_vx(int vx, int nw, bool nts, const StepTile& t, hipStream_t st)
{
    switch (vx) {
    case 1: return launch2_nw<T, SHIFT, 1>(nw, nts, t, st);
    case 2: return launch2_nw<T, SHIFT, 2>(nw, nts, t, st);
    default: return hipErrorInvalidValue;
    }
}

// dtype: 0 FP64, 1 FP32, 2 FP32-shifted (FP16 storage has no two-step form).
bool step2_shape_supported(int dtype, int vx, int nw)
{
    return dtype >= 0 && dtype <= 2 && (vx == 1 || vx == 2) && (nw == 12 || nw == 16);
}

// flags: LBM_TILE_NT_STORE (2) selects non-temporal stores.
hipError_t launch_step2(int dtype, int vx, int nw, int flags, const StepTile& t, hipStream_t st)
{
    if (!step2_shape_supported(dtype, vx, nw) || t.field) return hipErrorInvalidValue;
    const bool nts = (flags & 2) != 0;
    switch (dtype) {
    case 0: return launch2_vx<double, false>(vx, nw, nts, t, st);
    case 1: return launch2_vx<float, false>(vx, nw, nts, t, st);
    case 2: return launch2_vx<float, true>(vx, nw, nts, t, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
