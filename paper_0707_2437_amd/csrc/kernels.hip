// kernels.hip -- HIP kernels (gfx950) for the variable-speed-of-sound D2Q9
// lattice Boltzmann step (Buick & Cosgrove, Sec. 3 Eq. 5), in the pull
// storage described in internal.h.
//
// The step is bound by HBM bandwidth (9 reads + 9 writes per site, ~1 flop
// per byte), so there is no matrix-core work: the kernel is organised for
// coalesced row-contiguous traffic.
//
// Work decomposition of one step: every 64-lane wave owns a column strip of
// 64 * VX sites and marches down (or up) a chunk of h rows. For each row a
// lane loads, per link plane, a window of VX + 2 consecutive stored values:
// the pulled populations of its VX sites and of the sites just left and
// right of them (neighbouring lanes' windows overlap, so the overlap is
// served by the caches, not by HBM). It can therefore form the density of
// its own sites and of both x-neighbours itself, and the central-difference
// gradient (Sec. 4) needs no exchange between lanes: the y-neighbours'
// densities are the previous and next rows of the march, kept in
// registers. There is no LDS and no barrier; waves are independent. The
// loads of the next row are issued before the current row is relaxed and
// written (one row of prefetch). Only the two rows just outside a chunk are
// read twice (by the waves of the two chunks that share them); alternate
// chunks march in opposite directions so that both reads of a shared row
// happen at the start (or both at the end) of the two marches, close in
// time.
//
// Determinism: every site's arithmetic is the same code in the same order,
// whatever the tile shape or march direction, so results are bitwise
// independent of the tile. The build uses -ffp-contract=off; fused
// multiply-adds are written explicitly.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "step.h"

namespace lbm {

template <class T, bool SHIFT, int VX, int NW, int PF, bool NTS>
__global__ __launch_bounds__(64 * NW) void step_kernel(StepTile a, int ntiles)
{
    using C = typename CompT<T>::type;
    using K = KeepT<T, C>;
    constexpr int WV = VX + 2;  // window: columns x-1 .. x+VX
    using R = Pack<T, WV>;

    // XCD-aware tile order: consecutive blocks go round-robin over the 8
    // XCDs, so give each XCD a contiguous run of tiles. In row-band order
    // (LBM_TILE_ROWBAND) tiles run over the strip groups of a chunk first:
    // when the grid is larger than what is resident, each XCD then sweeps a
    // band of consecutive rows through memory (DRAM page locality), and the
    // boundary rows two vertically adjacent chunks share are read by
    // co-resident workgroups of one XCD (the second read hits its L2).
    // Otherwise tiles run over the chunks of a strip group first.
    const int nb = gridDim.x;  // a multiple of 8
    const int b = blockIdx.x;
    const int t = (b & 7) * (nb >> 3) + (b >> 3);
    if (t >= ntiles) return;
    const int ngroups = ntiles / a.nchunks;
    int group, chunk;
    if (a.rowband) {
        chunk = t / ngroups;
        group = t - chunk * ngroups;
    } else {
        group = t / a.nchunks;
        chunk = t - group * a.nchunks;
    }
    const int strip = group * NW + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const Geom g = a.g;
    const int x = strip * (64 * VX) + lane * VX;
    const int nv = min(VX, g.nx - x);
    if (nv <= 0) return;  // no barrier below: lanes past the edge simply leave
    const CoefC<C> k = coef_c<C>(a.c);
    const Centre<C> cn = centre_c<C>(a.c);
    const int ylo = chunk * a.h;
    const int yhi = min(ylo + a.h, g.ny);
    const int dir = (chunk & 1) ? -1 : 1;  // alternate chunks march upward
    const int ys = dir > 0 ? ylo : yhi - 1;
    const int nrow = yhi - ylo;

    const char* sb[9];
    char* dbase[9];
    plane_bases<T>(a.src, a.dst, g, sb, dbase);

    K da[9][VX], db[9][VX];        // populations of the current and next row (own columns)
    C wa[WV], wb[WV];              // densities of the current and next row, window columns
    C rprev[VX];                   // densities of the previous row, own columns
    R ra[9], rb[9];                // loads in flight (PF rows ahead)

    // Land a window row: populations of the own columns, densities of all
    // window columns (same summation order as every other code path).
    auto land = [&](const R (&v)[9], K (&d)[9][VX], C (&w)[WV]) {
        K tmp[9][WV];
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < WV; ++j) tmp[i][j] = keep_of<T, SHIFT, C>(v[i].v[j], i, cn);
#pragma unroll
        for (int j = 0; j < WV; ++j) w[j] = drho_of<T, SHIFT, C, WV>(tmp, j, cn);
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < VX; ++j) d[i][j] = tmp[i][j + 1];
    };

    auto collide_row = [&](int y, const K (&dc)[9][VX], const C (&wc)[WV], const C (&wn)[WV]) {
        Pack<T, VX> out[9];
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            // central differences at time t (Sec. 4); y +- 1 are the march's
            // next / previous rows in the order of the march direction
            // (undivided: the 1/2 is in the source coefficient)
            const C gx = wc[j + 2] - wc[j];
            const C up = wn[j + 1], dw = rprev[j];
            const C gy = dir > 0 ? up - dw : dw - up;
            C o[9];
            collide<T, SHIFT, C, VX>(dc, j, wc[j + 1], gx, gy, k, cn, o);
#pragma unroll
            for (int i = 0; i < 9; ++i) out[i].v[j] = from_d<T, SHIFT, C>(o[i], i, cn);
        }
        write_row<T, VX, NTS>(dbase, g, y, x, nv, out);
    };

    // March. Entering row y (the k-th of the chunk): row y's populations and
    // window densities are in registers, rprev holds the densities of the
    // row before it, and the loads of the next PF rows are in flight. Each
    // iteration lands row y + dir, issues the loads of row y + (PF+1) dir,
    // then relaxes and writes row y. The loop is unrolled by two so the
    // register sets alternate roles instead of being copied.
    {
        K dt[9][VX];
        C wt[WV];
        gather_raw<T, WV>(sb, g, ys - dir, x, ra);
        land(ra, dt, wt);
#pragma unroll
        for (int j = 0; j < VX; ++j) rprev[j] = wt[j + 1];
        gather_raw<T, WV>(sb, g, ys, x, ra);
        land(ra, da, wa);
    }
    if constexpr (PF >= 1) gather_raw<T, WV>(sb, g, ys + dir, x, ra);
    if constexpr (PF >= 2) {
        if (nrow >= 2) gather_raw<T, WV>(sb, g, ys + 2 * dir, x, rb);
    }
    auto advance = [&](int kk, K (&dc)[9][VX], K (&dn)[9][VX], C (&wc)[WV], C (&wn)[WV], R (&rl)[9]) {
        const int y = ys + dir * kk;
        if constexpr (PF == 0) gather_raw<T, WV>(sb, g, y + dir, x, rl);
        land(rl, dn, wn);
        if constexpr (PF >= 1) {
            if (kk + PF + 1 <= nrow) gather_raw<T, WV>(sb, g, y + (PF + 1) * dir, x, rl);
        }
        collide_row(y, dc, wc, wn);
#pragma unroll
        for (int j = 0; j < VX; ++j) rprev[j] = wc[j + 1];
    };
    // the raw buffer landed at step kk is ra for even kk when PF != 2
    int kk = 0;
    for (; kk + 1 < nrow; kk += 2) {
        advance(kk, da, db, wa, wb, ra);
        advance(kk + 1, db, da, wb, wa, PF == 2 ? rb : ra);
    }
    if (kk < nrow) advance(kk, da, db, wa, wb, ra);
}

// Vertical-stack form of the same step (see vstack_tile in step.h). Each
// workgroup takes one tile; all rows of a group are in flight together and
// tiles run over the strips of a row group first, dealt to the XCDs in
// chunks (xcd_tile), so the set of rows being streamed at any time stays
// one compact band. Each row is read (R + 2) / R times; the extra reads of
// the boundary rows are served by the caches.
// FIELD: a lattice with a c2 field (per-site source coefficients).
template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MinWaves<T>::value, 8))) void step_vstack_kernel(
    StepTile a, int ntiles)
{
    using C = typename CompT<T>::type;
    __shared__ C lds[NW][64 * VX];
    const int t = xcd_tile(blockIdx.x, gridDim.x, a.xcd_chunk);
    if (t >= ntiles) return;
    vstack_tile<T, SHIFT, VX, NW, NTS, FIELD>(a, a.src, a.dst, t % a.nstrips, t / a.nstrips, lds);
}

// ---------------------------------------------------------------------------
// Set-up and read-out kernels (one thread per element; not on the hot path).

__device__ __forceinline__ int wrapx2(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }  // x in [-n, 2n)

__device__ __constant__ int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ __constant__ int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

__device__ __forceinline__ double wt64(int i) { return wt<double>(i); }

// eqs is the equilibrium shift of the altered-equilibrium model (0 for
// Eq. 2): the moving populations gain w_i rho eqs, the rest population loses
// their sum, (1 - w_0) rho eqs.
__device__ __forceinline__ double eq_adjust(int i, double rho, double eqs)
{
    return i == 0 ? -(1.0 - wt64(0)) * rho * eqs : wt64(i) * rho * eqs;
}
// The model's equilibrium at rest, r_i = w_i + eq_adjust(i, 1): the centre
// of the shifted storage (Centre in step.h); w_i for Eq. 2.
__device__ __forceinline__ double centre64(int i, double eqs) { return wt64(i) + eq_adjust(i, 1.0, eqs); }
// Eq. 2 (with the model's shift), returned as feq_i - r_i (accurate for the
// shifted forms): eq_adjust is linear in rho, so its part is eq_adjust(rho - 1).
__device__ __forceinline__ double dfeq(int i, double rho, double ux, double uy, double eqs)
{
    const double eu = kEX[i] * ux + kEY[i] * uy;
    const double usq = ux * ux + uy * uy;
    return wt64(i) * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq)) + eq_adjust(i, rho - 1.0, eqs);
}
__device__ __forceinline__ double feq(int i, double rho, double ux, double uy, double eqs)
{
    const double eu = kEX[i] * ux + kEY[i] * uy;
    const double usq = ux * ux + uy * uy;
    return wt64(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq) + eq_adjust(i, rho, eqs);
}

template <class T, bool SHIFT> __device__ __forceinline__ T store_f64(double f, int i, double eqs)
{
    if constexpr (SHIFT) return (T)(f - centre64(i, eqs));
    else return (T)f;
}
template <class T, bool SHIFT> __device__ __forceinline__ double load_f64(T v, int i, double eqs)
{
    if constexpr (SHIFT) return (double)v + centre64(i, eqs);
    else return (double)v;
}

// Element (i, y, xx) of a 1-D launch over 9 * ny rows of `w` columns.
// Every element (i, y, col) of 9 * ny rows of w columns, by a grid-stride
// loop: a large lattice has more elements than one dispatch may have work
// items (the count is 32-bit), so the grid is capped (plane_rows_grid) and
// each thread visits every (grid size)-th element.
template <class F> __device__ __forceinline__ void for_each_row_elem(const Geom& g, int w, F&& f)
{
    const long long n = 9LL * g.ny * w, stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const long long row = q / w;
        const int col = (int)(q - row * w);
        const int i = (int)(row / g.ny);
        const int y = (int)(row - (long long)i * g.ny);
        f(i, y, col);
    }
}

// S_i(x, y) = feq_i(rho, u at (x + e_i, y + e_i)) for x in [-2, nx + 1] (the
// ghost columns included): the pulled gather of the first step then sees
// f_i(x, 0) = feq_i(x).
template <class T, bool SHIFT>
__global__ void init_kernel(T* __restrict__ s, Geom g, const double* __restrict__ rho, const double* __restrict__ ux,
                            const double* __restrict__ uy, double eqs)
{
    for_each_row_elem(g, g.nx + 4, [&](int i, int y, int col) {
        const int xx = col - 2;  // -2 .. nx + 1
        const int sx = wrapx2(xx + kEX[i], g.nx), sy = wrapy(y + kEY[i], g.ny);
        const long long q = (long long)sy * g.nx + sx;
        const double r = rho ? rho[q] : 1.0, vx = ux ? ux[q] : 0.0, vy = uy ? uy[q] : 0.0;
        T v;
        if constexpr (SHIFT) v = (T)dfeq(i, r, vx, vy, eqs);
        else v = (T)feq(i, r, vx, vy, eqs);
        s[i * g.ps + (long long)y * g.rs + g.off + xx] = v;
    });
}

// S_i(x) = f_i(x + e_i), x in [-2, nx + 1], from a canonical FP64 array [9][ny][nx].
template <class T, bool SHIFT>
__global__ void set_f_kernel(T* __restrict__ s, Geom g, const double* __restrict__ f, double eqs)
{
    for_each_row_elem(g, g.nx + 4, [&](int i, int y, int col) {
        const int xx = col - 2;  // -2 .. nx + 1
        const int sx = wrapx2(xx + kEX[i], g.nx), sy = wrapy(y + kEY[i], g.ny);
        s[i * g.ps + (long long)y * g.rs + g.off + xx] =
            store_f64<T, SHIFT>(f[((long long)i * g.ny + sy) * g.nx + sx], i, eqs);
    });
}

// f_i(x) = S_i(x - e_i) into a canonical FP64 array [9][ny][nx].
template <class T, bool SHIFT>
__global__ void get_f_kernel(const T* __restrict__ s, Geom g, double* __restrict__ f, double eqs)
{
    for_each_row_elem(g, g.nx, [&](int i, int y, int xx) {
        const int sy = wrapy(y - kEY[i], g.ny), sx = wrapx2(xx - kEX[i], g.nx);
        f[((long long)i * g.ny + y) * g.nx + xx] =
            load_f64<T, SHIFT>(s[i * g.ps + (long long)sy * g.rs + g.off + sx], i, eqs);
    });
}

// f_i at n listed sites into out[n][9].
template <class T, bool SHIFT>
__global__ void sample_f_kernel(const T* __restrict__ s, Geom g, int n, const int* __restrict__ xy,
                                double* __restrict__ out, double eqs)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 9 * n) return;
    const int k = q / 9, i = q - 9 * k;
    const int x = xy[2 * k], y = xy[2 * k + 1];
    const int sy = wrapy(y - kEY[i], g.ny), sx = wrapx2(x - kEX[i], g.nx);
    out[q] = load_f64<T, SHIFT>(s[i * g.ps + (long long)sy * g.rs + g.off + sx], i, eqs);
}

// Moments (Eq. 3) of f(x, t) in FP64, optional fields, and per-block
// partial sums of (rho - 1, j_x, j_y) for the conservation totals.
constexpr int kRedThreads = 256;
constexpr int kRedWaves = kRedThreads / 64;

// Sum over the 64 lanes of a wave by a butterfly of cross-lane exchanges
// (no LDS, no barrier). The exchange pattern is fixed, so every lane's sum
// is the same from run to run; the callers use lane 0's.
__device__ inline double wave_sum(double v)
{
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// The three sums of a block: each wave's by wave_sum, then the kRedWaves
// wave sums in wave order, written by threads 0..2 to out[0..2].
__device__ inline void block_sum3(double a, double b, double c, double* __restrict__ out)
{
    __shared__ double red[3][kRedWaves];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int wave = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
        red[2][wave] = c;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = red[threadIdx.x][0];
        for (int w = 1; w < kRedWaves; ++w) t += red[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
}

template <class T, bool SHIFT>
__global__ __launch_bounds__(kRedThreads) void moments_kernel(const T* __restrict__ s, Geom g, double* __restrict__ rho,
                                                              double* __restrict__ ux, double* __restrict__ uy,
                                                              double* __restrict__ partials)
{
    const long long n = (long long)g.nx * g.ny;
    double dr = 0.0, jx = 0.0, jy = 0.0;
    // grid-stride over sites, fixed order per thread (the block count depends
    // only on the lattice size, so the sums are deterministic)
    for (long long q = (long long)blockIdx.x * kRedThreads + threadIdx.x; q < n;
         q += (long long)gridDim.x * kRedThreads) {
        const int y = (int)(q / g.nx), x = (int)(q - (long long)y * g.nx);
        // Shifted forms store g_i = f_i - w_i; since sum_i w_i e_i = 0 the
        // momentum is sum_i g_i e_i as well, and rho = 1 + sum_i g_i.
        double vsum = 0.0, sx = 0.0, sy2 = 0.0;
        for (int i = 0; i < 9; ++i) {
            const int cy = wrapy(y - kEY[i], g.ny), cx = wrapx2(x - kEX[i], g.nx);
            const double v = (double)s[i * g.ps + (long long)cy * g.rs + g.off + cx];
            vsum += v;
            sx += v * kEX[i];
            sy2 += v * kEY[i];
        }
        const double r = SHIFT ? 1.0 + vsum : vsum;
        dr += SHIFT ? vsum : vsum - 1.0;
        jx += sx;
        jy += sy2;
        if (rho) rho[q] = r;
        if (ux) ux[q] = sx / r;
        if (uy) uy[q] = sy2 / r;
    }
    block_sum3(dr, jx, jy, partials + (long long)blockIdx.x * 3);
}

// Fixed-order reduction of nparts partial triples; out = {N + sum drho, sum jx, sum jy}.
__global__ __launch_bounds__(kRedThreads) void reduce_partials_kernel(const double* __restrict__ partials, int nparts,
                                                                      double nsites, double* __restrict__ out)
{
    __shared__ double sums[3];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nparts; p += kRedThreads)
        for (int c = 0; c < 3; ++c) acc[c] += partials[(long long)p * 3 + c];
    block_sum3(acc[0], acc[1], acc[2], sums);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = nsites + sums[0];
        out[1] = sums[1];
        out[2] = sums[2];
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers.

template <class T, bool SHIFT, int VX, int NW, int PF, bool NTS>
static hipError_t launch_step_t(const StepTile& t, hipStream_t st)
{
    const int ntiles = t.nstrips * t.nchunks;  // nstrips counts groups of NW strips
    const int grid = (ntiles + 7) / 8 * 8;
    if (!grid_fits(grid, 64 * NW)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((step_kernel<T, SHIFT, VX, NW, PF, NTS>), dim3(grid), dim3(64 * NW), 0, st, t, ntiles);
    return hipGetLastError();
}

// flags: LBM_TILE_PREFETCH (1), LBM_TILE_NT_STORE (2), LBM_TILE_ROWBAND (4,
// a runtime switch), LBM_TILE_PREFETCH2 (8: two rows ahead).
template <class T, bool SHIFT, int VX, int NW>
static hipError_t launch_flags(int flags, const StepTile& t, hipStream_t st)
{
    const int pf = (flags & 8) ? 2 : (flags & 1);
    const bool nts = (flags & 2) != 0;
    switch (pf * 2 + (nts ? 1 : 0)) {
    case 0: return launch_step_t<T, SHIFT, VX, NW, 0, false>(t, st);
    case 1: return launch_step_t<T, SHIFT, VX, NW, 0, true>(t, st);
    case 2: return launch_step_t<T, SHIFT, VX, NW, 1, false>(t, st);
    case 3: return launch_step_t<T, SHIFT, VX, NW, 1, true>(t, st);
    case 4: return launch_step_t<T, SHIFT, VX, NW, 2, false>(t, st);
    default: return launch_step_t<T, SHIFT, VX, NW, 2, true>(t, st);
    }
}

template <class T, bool SHIFT, int VX, int NW>
static hipError_t launch_vstack_t(int flags, const StepTile& t, hipStream_t st)
{
    const int ntiles = t.nstrips * t.nchunks;  // strips x row groups of NW - 2 rows
    const int q = t.xcd_chunk > 0 ? 8 * t.xcd_chunk : 8;
    const int grid = (ntiles + q - 1) / q * q;
    if (!grid_fits(grid, 64 * NW)) return hipErrorInvalidConfiguration;
    const dim3 gd(grid), bd(64 * NW);
    if (t.field) {
        if (flags & 2) hipLaunchKernelGGL((step_vstack_kernel<T, SHIFT, VX, NW, true, true>), gd, bd, 0, st, t, ntiles);
        else hipLaunchKernelGGL((step_vstack_kernel<T, SHIFT, VX, NW, false, true>), gd, bd, 0, st, t, ntiles);
    } else {
        if (flags & 2) hipLaunchKernelGGL((step_vstack_kernel<T, SHIFT, VX, NW, true, false>), gd, bd, 0, st, t, ntiles);
        else hipLaunchKernelGGL((step_vstack_kernel<T, SHIFT, VX, NW, false, false>), gd, bd, 0, st, t, ntiles);
    }
    return hipGetLastError();
}

template <class T, bool SHIFT, int VX>
static hipError_t launch_nw(int nw, int flags, const StepTile& t, hipStream_t st)
{
    if (flags & 16) {
        switch (nw) {
        case 4: return launch_vstack_t<T, SHIFT, VX, 4>(flags, t, st);
        case 8: return launch_vstack_t<T, SHIFT, VX, 8>(flags, t, st);
        case 16: return launch_vstack_t<T, SHIFT, VX, 16>(flags, t, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (nw) {
    case 1: return launch_flags<T, SHIFT, VX, 1>(flags, t, st);
    case 4: return launch_flags<T, SHIFT, VX, 4>(flags, t, st);
    default: return hipErrorInvalidValue;
    }
}

template <class T, bool SHIFT>
static hipError_t launch_vx(int vx, int nw, int flags, const StepTile& t, hipStream_t st)
{
    switch (vx) {
    case 1: return launch_nw<T, SHIFT, 1>(nw, flags, t, st);
    case 2: return launch_nw<T, SHIFT, 2>(nw, flags, t, st);
    case 4: return launch_nw<T, SHIFT, 4>(nw, flags, t, st);
    default: return hipErrorInvalidValue;
    }
}

bool step_shape_supported(int dtype, int vx, int nw, int flags)
{
    if (dtype < 0 || dtype > 3 || !(vx == 1 || vx == 2 || vx == 4)) return false;
    if (flags & 16) return nw == 4 || nw == 8 || nw == 16;
    return nw == 1 || nw == 4;
}

hipError_t launch_step(int dtype, int vx, int nw, int flags, const StepTile& t, hipStream_t st)
{
    if (!step_shape_supported(dtype, vx, nw, flags)) return hipErrorInvalidValue;
    if (t.field && !(flags & 16)) return hipErrorInvalidValue;  // c2 fields: vertical-stack kernels only
    switch (dtype) {
    case 0: return launch_vx<double, false>(vx, nw, flags, t, st);
    case 1: return launch_vx<float, false>(vx, nw, flags, t, st);
    case 2: return launch_vx<float, true>(vx, nw, flags, t, st);
    case 3: return launch_vx<_Float16, true>(vx, nw, flags, t, st);
    }
    return hipErrorInvalidValue;
}

// Fig. 1 boundaries, after the step from time t into `s` (which then holds
// the post-collision populations S_i(x) = f*_i(x, t)): the sites of columns
// 0 and nx - 1 emit the equilibrium at rest at rho_in and 1 in place of
// their collision, and a population that crosses the cut periodic seam
// carries the equilibrium of the column it enters. One thread per (plane,
// row, column) over columns 0, nx - 1 and their ghost images nx and -1
// (read in place of the wrap by the FP16 kernels; padding otherwise).
template <class T, bool SHIFT>
__global__ void xbc_kernel(T* __restrict__ s, Geom g, double rho_in, double eqs)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 36LL * g.ny) return;
    const int k = (int)(q & 3);
    const long long row = q >> 2;
    const int i = (int)(row / g.ny), y = (int)(row - (long long)i * g.ny);
    const bool inlet = k == 0 || k == 2;  // column 0, or its image nx
    const int col = k == 0 ? 0 : (k == 1 ? g.nx - 1 : (k == 2 ? g.nx : -1));
    const bool crosses = inlet ? kEX[i] < 0 : kEX[i] > 0;
    const double rho = inlet != crosses ? rho_in : 1.0;
    T v;
    if constexpr (SHIFT) v = (T)dfeq(i, rho, 0.0, 0.0, eqs);
    else v = (T)feq(i, rho, 0.0, 0.0, eqs);
    s[i * g.ps + (long long)y * g.rs + g.off + col] = v;
}

hipError_t launch_xbc(int dtype, void* s, const Geom& g, double rho_in, double eqs, hipStream_t st)
{
    const dim3 grid((unsigned)((36LL * g.ny + 255) / 256));
    switch (dtype) {
    case 0: hipLaunchKernelGGL((xbc_kernel<double, false>), grid, dim3(256), 0, st, (double*)s, g, rho_in, eqs); break;
    case 1: hipLaunchKernelGGL((xbc_kernel<float, false>), grid, dim3(256), 0, st, (float*)s, g, rho_in, eqs); break;
    case 2: hipLaunchKernelGGL((xbc_kernel<float, true>), grid, dim3(256), 0, st, (float*)s, g, rho_in, eqs); break;
    case 3: hipLaunchKernelGGL((xbc_kernel<_Float16, true>), grid, dim3(256), 0, st, (_Float16*)s, g, rho_in, eqs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// c2 field -> per-site source coefficients in compute precision C; the
// pitch padding (x >= nx) is zero.
template <class C>
__global__ void field_kernel(C* __restrict__ field, int nx, int ny, int fpitch, const double* __restrict__ c2)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)ny * fpitch) return;
    const int y = (int)(k / fpitch), x = (int)(k % fpitch);
    field[k] = x < nx ? (C)source_as1(c2[(size_t)y * nx + x]) : C(0);
}

hipError_t launch_field(int dtype, void* field, int nx, int ny, int fpitch, const double* c2, hipStream_t st)
{
    const long long n = (long long)ny * fpitch;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (dtype == 0) hipLaunchKernelGGL(field_kernel<double>, grid, dim3(256), 0, st, (double*)field, nx, ny, fpitch, c2);
    else hipLaunchKernelGGL(field_kernel<float>, grid, dim3(256), 0, st, (float*)field, nx, ny, fpitch, c2);
    return hipGetLastError();
}

// Blocks of 256 for the set-up kernels' grid-stride loops over 9 * ny rows of
// nx + extra elements: one element per thread up to 2^20 blocks (2^28 work
// items, well inside the 32-bit dispatch size).
static dim3 plane_rows_grid(const Geom& g, int extra)
{
    const long long n = 9LL * g.ny * (g.nx + extra);
    const long long b = (n + 255) / 256;
    return dim3((unsigned)(b < (1LL << 20) ? b : (1LL << 20)));
}

#define LBM_DISPATCH(dtype, CALL)                                  \
    switch (dtype) {                                               \
    case 0: { using T = double; constexpr bool S = false; CALL; }  \
    case 1: { using T = float; constexpr bool S = false; CALL; }   \
    case 2: { using T = float; constexpr bool S = true; CALL; }    \
    case 3: { using T = _Float16; constexpr bool S = true; CALL; } \
    default: return hipErrorInvalidValue;                          \
    }

hipError_t launch_init(int dtype, void* s, const Geom& g, const double* rho, const double* ux, const double* uy,
                       double eqs, hipStream_t st)
{
    LBM_DISPATCH(dtype, {
        hipLaunchKernelGGL((init_kernel<T, S>), plane_rows_grid(g, 4), dim3(256), 0, st, (T*)s, g, rho, ux, uy, eqs);
        return hipGetLastError();
    })
}

hipError_t launch_set_f(int dtype, void* s, const Geom& g, const double* f, double eqs, hipStream_t st)
{
    LBM_DISPATCH(dtype, {
        hipLaunchKernelGGL((set_f_kernel<T, S>), plane_rows_grid(g, 4), dim3(256), 0, st, (T*)s, g, f, eqs);
        return hipGetLastError();
    })
}

hipError_t launch_get_f(int dtype, const void* s, const Geom& g, double* f, double eqs, hipStream_t st)
{
    LBM_DISPATCH(dtype, {
        hipLaunchKernelGGL((get_f_kernel<T, S>), plane_rows_grid(g, 0), dim3(256), 0, st, (const T*)s, g, f, eqs);
        return hipGetLastError();
    })
}

hipError_t launch_sample_f(int dtype, const void* s, const Geom& g, int n, const int* xy, double* out, double eqs,
                           hipStream_t st)
{
    const dim3 grid((unsigned)((9LL * n + 255) / 256));
    LBM_DISPATCH(dtype, {
        hipLaunchKernelGGL((sample_f_kernel<T, S>), grid, dim3(256), 0, st, (const T*)s, g, n, xy, out, eqs);
        return hipGetLastError();
    })
}

int moments_blocks(const Geom& g)
{
    const long long n = (long long)g.nx * g.ny;
    const long long nb = (n + kRedThreads - 1) / kRedThreads;
    return (int)(nb < 1024 ? nb : 1024);
}

hipError_t launch_moments(int dtype, const void* s, const Geom& g, double* rho, double* ux, double* uy,
                          double* partials, double* totals, hipStream_t st)
{
    const int nb = moments_blocks(g);
    hipError_t e = hipSuccess;
    switch (dtype) {
    case 0:
        hipLaunchKernelGGL((moments_kernel<double, false>), dim3(nb), dim3(kRedThreads), 0, st, (const double*)s, g,
                           rho, ux, uy, partials);
        break;
    case 1:
        hipLaunchKernelGGL((moments_kernel<float, false>), dim3(nb), dim3(kRedThreads), 0, st, (const float*)s, g,
                           rho, ux, uy, partials);
        break;
    case 2:
        hipLaunchKernelGGL((moments_kernel<float, true>), dim3(nb), dim3(kRedThreads), 0, st, (const float*)s, g, rho,
                           ux, uy, partials);
        break;
    case 3:
        hipLaunchKernelGGL((moments_kernel<_Float16, true>), dim3(nb), dim3(kRedThreads), 0, st,
                           (const _Float16*)s, g, rho, ux, uy, partials);
        break;
    default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kRedThreads), 0, st, partials, nb,
                       (double)g.nx * (double)g.ny, totals);
    return hipGetLastError();
}

}  // namespace lbm
