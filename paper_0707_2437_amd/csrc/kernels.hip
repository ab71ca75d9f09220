// kernels.hip -- HIP kernels (gfx950) for the variable-speed-of-sound D2Q9
// lattice Boltzmann step (Buick & Cosgrove, Sec. 3 Eq. 5), in the pull
// storage described in internal.h.
//
// The step is bound by HBM bandwidth (9 reads + 9 writes per site, ~1 flop
// per byte), so there is no matrix-core work: the kernel is organised for
// coalesced row-contiguous traffic.
//
// Work decomposition of one step: the lattice is cut into column strips of
// W = 64 * NW * VX sites and row chunks of h rows; one workgroup marches down
// one (strip, chunk) tile row by row. For the current row it gathers the
// nine pulled populations of every site with contiguous (possibly
// one-element-misaligned) vector loads, keeps them in registers, and puts
// the site density into an LDS ring so that the central-difference gradient
// (Sec. 4) can read the x-neighbours; the y-neighbours' densities are the
// previous and next rows of the march, kept in registers. Two lanes also
// gather the density of the columns just left and right of the strip.
// Every S value is read from HBM once per tile; only the two extra rows of a
// chunk (the y-halo of the gradient) are read twice.
//
// Determinism: every site's arithmetic is the same code in the same order,
// whatever the tile shape, so results are bitwise independent of the tile
// (the density of a halo column is computed exactly as its owner computes
// it). The build uses -ffp-contract=off; fused multiply-adds are written
// explicitly.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace lbm {

template <class T> struct CompT { using type = float; };
template <> struct CompT<double> { using type = double; };

// Lattice weights (Sec. 2) in compute precision.
template <class C> __device__ __forceinline__ C wt(int i)
{
    return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}

__device__ __forceinline__ int wrapy(int r, int ny) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); }

// Stored value -> d_i = f_i - w_i in compute precision, and back.
template <class T, bool SHIFT, class C> __device__ __forceinline__ C to_d(T v, int i)
{
    if constexpr (SHIFT) return (C)v;
    else return (C)v - wt<C>(i);
}
template <class T, bool SHIFT, class C> __device__ __forceinline__ T from_d(C d, int i)
{
    if constexpr (SHIFT) return (T)d;
    else return (T)(wt<C>(i) + d);
}

template <class T, int VX> struct Pack { T v[VX]; };

// Memory is addressed as a per-plane base pointer (uniform, computed once
// per workgroup, held in scalar registers) plus a 32-bit byte offset
// (row offset + lane offset), which maps to SGPR-based global loads and
// stores. Only element alignment is assumed: planes 1, 3, 5-8 are read one
// element off a vector boundary, and gfx950 executes such dwordx2/x4 loads
// directly. A plane is limited to 4 GiB (checked at create).
template <class T, int VX> __device__ __forceinline__ Pack<T, VX> ld_vec(const char* base, unsigned byte_off)
{
    Pack<T, VX> r;
    __builtin_memcpy(&r, base + (size_t)byte_off, sizeof(r));
    return r;
}

// Registers hold the populations of two rows. FP32/FP64 storage is kept
// as d_i = f_i - w_i in compute precision; FP16 storage is kept raw (half
// the registers) and converted where it is used.
template <class T, class C> using KeepT = typename std::conditional<(sizeof(T) < sizeof(C)), T, C>::type;

template <class T, bool SHIFT, class C> __device__ __forceinline__ KeepT<T, C> keep_of(T v, int i)
{
    if constexpr (sizeof(T) < sizeof(C)) return v;
    else return to_d<T, SHIFT, C>(v, i);
}
template <class T, bool SHIFT, class C> __device__ __forceinline__ C d_of(KeepT<T, C> v, int i)
{
    if constexpr (sizeof(T) < sizeof(C)) return to_d<T, SHIFT, C>(v, i);
    else return v;
}

// Gather f_i(x + j, r) = S_i(x + j - e_ix, r - e_iy), j < VX.
// Links (Sec. 2): e_0 (0,0); e_1 (1,0); e_2 (0,1); e_3 (-1,0); e_4 (0,-1);
// e_5 (1,1); e_6 (-1,1); e_7 (-1,-1); e_8 (1,-1).
// pb[i] points at column -1 of row 0 of plane i, so the byte offset of
// column x - e_ix in row q is (q * pitch + x + 1 - e_ix) * sizeof(T) >= 0.
template <class T, bool SHIFT, int VX, class C>
__device__ __forceinline__ void gather(const char* const (&pb)[9], const Geom& g, int r, int x, KeepT<T, C> d[9][VX])
{
    constexpr unsigned es = sizeof(T);
    const unsigned om = (unsigned)wrapy(r - 1, g.ny) * (unsigned)g.pitch * es;  // source row r - 1 (e_iy = +1)
    const unsigned o0 = (unsigned)wrapy(r, g.ny) * (unsigned)g.pitch * es;      // source row r     (e_iy =  0)
    const unsigned op = (unsigned)wrapy(r + 1, g.ny) * (unsigned)g.pitch * es;  // source row r + 1 (e_iy = -1)
    const unsigned xm = (unsigned)x * es, x0 = xm + es, xp = xm + 2 * es;       // columns x-1, x, x+1
    Pack<T, VX> v[9];
    v[0] = ld_vec<T, VX>(pb[0], o0 + x0);
    v[1] = ld_vec<T, VX>(pb[1], o0 + xm);
    v[2] = ld_vec<T, VX>(pb[2], om + x0);
    v[3] = ld_vec<T, VX>(pb[3], o0 + xp);
    v[4] = ld_vec<T, VX>(pb[4], op + x0);
    v[5] = ld_vec<T, VX>(pb[5], om + xm);
    v[6] = ld_vec<T, VX>(pb[6], om + xp);
    v[7] = ld_vec<T, VX>(pb[7], op + xp);
    v[8] = ld_vec<T, VX>(pb[8], op + xm);
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < VX; ++j) d[i][j] = keep_of<T, SHIFT, C>(v[i].v[j], i);
}

// delta rho = sum_i d_i (Eq. 3), one fixed order for every code path.
template <class T, bool SHIFT, class C, int VX> __device__ __forceinline__ C drho_of(const KeepT<T, C> d[9][VX], int j)
{
    auto D = [&](int i) { return d_of<T, SHIFT, C>(d[i][j], i); };
    return (((D(0) + D(1)) + (D(2) + D(3))) + ((D(4) + D(5)) + (D(6) + D(7)))) + D(8);
}

template <class C> struct CoefC {
    C om1, wo0, wo1, wo2, as1, as2;
};

template <class C> __device__ __forceinline__ CoefC<C> coef_c(const Coef& k)
{
    return CoefC<C>{(C)k.om1, (C)k.wo0, (C)k.wo1, (C)k.wo2, (C)k.as1, (C)k.as2};
}

// Fused multiply-add in the compute precision (the only FMAs the build emits).
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class C> __device__ __forceinline__ C recip(C r) { return C(1) / r; }
template <> __device__ __forceinline__ float recip<float>(float r) { return __builtin_amdgcn_rcpf(r); }

// Eq. 5 right-hand side in delta form for one site.
//   rho = 1 + drho, u = j / rho (Eq. 3)
//   feq_i - w_i = w_i [drho + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)]      (Eq. 2)
//   d*_i = d_i - (d_i - (feq_i - w_i))/tau + 3 w_i alpha (e_i . G)      (Eq. 5)
// For a link pair (i, opp) with e_opp = -e_i, write A = drho - 3/2 rho u.u,
// sym = A + 9/2 rho (e.u)^2, P = om w sym, Q = om w 3 rho (e.u) + 3 w alpha (e.G):
//   d*_i = (1 - om) d_i + P + Q,  d*_opp = (1 - om) d_opp + P - Q.
template <class T, bool SHIFT, class C, int VX>
__device__ __forceinline__ void collide(const KeepT<T, C> dk[9][VX], int j, C drho, C gx, C gy, const CoefC<C>& k,
                                        C o[9])
{
    C d[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = d_of<T, SHIFT, C>(dk[i][j], i);
    const C jx = ((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7]);
    const C jy = ((d[2] - d[4]) + (d[5] - d[8])) + (d[6] - d[7]);
    const C rho = C(1) + drho;
    const C ir = recip<C>(rho);
    const C ux = jx * ir, uy = jy * ir;
    const C usq = fmac(ux, ux, uy * uy);
    const C A = fmac(C(-1.5) * rho, usq, drho);
    const C r45 = C(4.5) * rho, r3 = C(3) * rho;
    o[0] = fmac(k.om1, d[0], k.wo0 * A);
    auto pair = [&](int i, int io, C eu, C eg, C wo, C as) {
        const C P = wo * fmac(r45, eu * eu, A);
        const C Q = fmac(as, eg, wo * (r3 * eu));
        o[i] = fmac(k.om1, d[i], P + Q);
        o[io] = fmac(k.om1, d[io], P - Q);
    };
    pair(1, 3, ux, gx, k.wo1, k.as1);
    pair(2, 4, uy, gy, k.wo1, k.as1);
    pair(5, 7, ux + uy, gx + gy, k.wo2, k.as2);
    pair(6, 8, uy - ux, gy - gx, k.wo2, k.as2);
}

template <class T, bool SHIFT, int VX, int NW>
__global__ __launch_bounds__(64 * NW) void step_kernel(StepTile a, int ntiles)
{
    using C = typename CompT<T>::type;
    using K = KeepT<T, C>;
    constexpr int NT = 64 * NW;
    constexpr int W = NT * VX;
    __shared__ C ring[4][W + 2];  // delta rho of rows; [0] and [wv+1] are the halo columns

    // XCD-aware tile order: consecutive blocks go round-robin over the 8
    // XCDs, so give each XCD a contiguous run of tiles (vertically adjacent
    // chunks of a strip share their halo rows in that XCD's L2).
    const int nb = gridDim.x;  // a multiple of 8
    const int b = blockIdx.x;
    const int t = (b & 7) * (nb >> 3) + (b >> 3);
    if (t >= ntiles) return;
    const int strip = t / a.nchunks;
    const int chunk = t - strip * a.nchunks;
    const Geom g = a.g;
    const CoefC<C> k = coef_c<C>(a.c);
    const int xs = strip * W;
    const int wv = min(W, g.nx - xs);
    const int y0 = chunk * a.h;
    const int y1 = min(y0 + a.h, g.ny);
    const int tid = threadIdx.x;
    const int lx = tid * VX;
    const int x = xs + lx;
    const int nv = min(VX, wv - lx);
    // per-plane bases: source at column -1, destination at column 0
    const char* sb[9];
    char* dbase[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        sb[i] = (const char*)a.src + ((long long)i * g.plane + g.off - 1) * (long long)sizeof(T);
        dbase[i] = (char*)a.dst + ((long long)i * g.plane + g.off) * (long long)sizeof(T);
    }

    const bool hl = tid == NT - 1, hr = tid == NT - 2;
    const int xh = hl ? (xs == 0 ? g.nx - 1 : xs - 1) : (xs + wv == g.nx ? 0 : xs + wv);
    const int hpos = hl ? 0 : wv + 1;

    K da[9][VX], db[9][VX];
    C rp[VX], rc[VX], rn[VX];

    // Density of row r at this lane's columns into rr[] and the ring, and of
    // the halo column (two lanes).
    auto gather_row = [&](int r, K (&d)[9][VX], C (&rr)[VX], bool to_ring) {
        if (nv > 0) {
            gather<T, SHIFT, VX, C>(sb, g, r, x, d);
#pragma unroll
            for (int j = 0; j < VX; ++j) {
                rr[j] = drho_of<T, SHIFT, C, VX>(d, j);
                if (to_ring && j < nv) ring[r & 3][lx + 1 + j] = rr[j];
            }
        }
        if (to_ring && (hl || hr)) {
            K h[9][1];
            gather<T, SHIFT, 1, C>(sb, g, r, xh, h);
            ring[r & 3][hpos] = drho_of<T, SHIFT, C, 1>(h, 0);
        }
    };

    // Collide row y (populations dc) and write it.
    auto collide_row = [&](int y, const K (&dc)[9][VX]) {
        if (nv <= 0) return;
        const C* rr = ring[y & 3];
        Pack<T, VX> out[9];
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            // central differences at time t (Sec. 4)
            const C gx = C(0.5) * (rr[lx + j + 2] - rr[lx + j]);
            const C gy = C(0.5) * (rn[j] - rp[j]);
            C o[9];
            collide<T, SHIFT, C, VX>(dc, j, rc[j], gx, gy, k, o);
#pragma unroll
            for (int i = 0; i < 9; ++i) out[i].v[j] = from_d<T, SHIFT, C>(o[i], i);
        }
        constexpr unsigned es = sizeof(T);
        const unsigned ro = (unsigned)y * (unsigned)g.pitch * es;  // row y, column 0
        const unsigned lo = ro + (unsigned)x * es;
        if (nv == VX) {
#pragma unroll
            for (int i = 0; i < 9; ++i) __builtin_memcpy(dbase[i] + (size_t)lo, &out[i], sizeof(out[i]));
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i)
#pragma unroll
                for (int j = 0; j < VX; ++j)
                    if (j < nv) __builtin_memcpy(dbase[i] + (size_t)(lo + j * es), &out[i].v[j], es);
        }
        // ghost columns: -1 holds column nx-1, nx holds column 0
        const int jl = g.nx - 1 - x;
        if (jl >= 0 && jl < nv) {
#pragma unroll
            for (int j = 0; j < VX; ++j)
                if (j == jl)
#pragma unroll
                    for (int i = 0; i < 9; ++i) __builtin_memcpy(dbase[i] + (size_t)ro - es, &out[i].v[j], es);
        }
        if (x == 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                __builtin_memcpy(dbase[i] + (size_t)(ro + (unsigned)g.nx * es), &out[i].v[0], es);
        }
    };

    // March: entering row y, the populations of row y are in registers,
    // rp/rc hold the densities of rows y-1 and y, and ring[y & 3] holds
    // row y's densities with its halo.
    gather_row(y0 - 1, db, rp, false);
    gather_row(y0, da, rc, true);
    auto advance = [&](int y, K (&dc)[9][VX], K (&dn)[9][VX]) {
        gather_row(y + 1, dn, rn, true);
        __syncthreads();
        collide_row(y, dc);
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            rp[j] = rc[j];
            rc[j] = rn[j];
        }
    };
    int y = y0;
    for (; y + 1 < y1; y += 2) {
        advance(y, da, db);
        advance(y + 1, db, da);
    }
    if (y < y1) advance(y, da, db);
}

// ---------------------------------------------------------------------------
// Set-up and read-out kernels (one thread per element; not on the hot path).

__device__ __forceinline__ int wrapx(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

__device__ __constant__ int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ __constant__ int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

__device__ __forceinline__ double wt64(int i) { return wt<double>(i); }

// Eq. 2, returned as feq_i - w_i (accurate for the shifted forms).
__device__ __forceinline__ double dfeq(int i, double rho, double ux, double uy)
{
    const double eu = kEX[i] * ux + kEY[i] * uy;
    const double usq = ux * ux + uy * uy;
    return wt64(i) * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
}
__device__ __forceinline__ double feq(int i, double rho, double ux, double uy)
{
    const double eu = kEX[i] * ux + kEY[i] * uy;
    const double usq = ux * ux + uy * uy;
    return wt64(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
}

template <class T, bool SHIFT> __device__ __forceinline__ T store_f64(double f, int i)
{
    if constexpr (SHIFT) return (T)(f - wt64(i));
    else return (T)f;
}
template <class T, bool SHIFT> __device__ __forceinline__ double load_f64(T v, int i)
{
    if constexpr (SHIFT) return (double)v + wt64(i);
    else return (double)v;
}

// Element (i, y, xx) of a 1-D launch over 9 * ny rows of `w` columns.
struct RowIdx {
    int i, y, col;
    bool ok;
};
__device__ __forceinline__ RowIdx row_idx(const Geom& g, int w)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    RowIdx r;
    const long long row = q / w;
    r.ok = row < 9LL * g.ny;
    r.col = (int)(q - row * w);
    r.i = (int)(row / g.ny);
    r.y = (int)(row - (long long)r.i * g.ny);
    return r;
}

// S_i(x, y) = feq_i(rho, u at (x + e_i, y + e_i)) for x in [-1, nx]:
// the pulled gather of the first step then sees f_i(x, 0) = feq_i(x).
template <class T, bool SHIFT>
__global__ void init_kernel(T* __restrict__ s, Geom g, const double* __restrict__ rho, const double* __restrict__ ux,
                            const double* __restrict__ uy)
{
    const RowIdx ri = row_idx(g, g.nx + 2);
    if (!ri.ok) return;
    const int i = ri.i, y = ri.y, xx = ri.col - 1;  // -1 .. nx
    const int sx = wrapx(xx + kEX[i], g.nx), sy = wrapy(y + kEY[i], g.ny);
    const long long q = (long long)sy * g.nx + sx;
    const double r = rho ? rho[q] : 1.0, vx = ux ? ux[q] : 0.0, vy = uy ? uy[q] : 0.0;
    T v;
    if constexpr (SHIFT) v = (T)dfeq(i, r, vx, vy);
    else v = (T)feq(i, r, vx, vy);
    s[i * g.plane + (long long)y * g.pitch + g.off + xx] = v;
}

// S_i(x) = f_i(x + e_i) from a canonical FP64 array [9][ny][nx].
template <class T, bool SHIFT> __global__ void set_f_kernel(T* __restrict__ s, Geom g, const double* __restrict__ f)
{
    const RowIdx ri = row_idx(g, g.nx + 2);
    if (!ri.ok) return;
    const int i = ri.i, y = ri.y, xx = ri.col - 1;  // -1 .. nx
    const int sx = wrapx(xx + kEX[i], g.nx), sy = wrapy(y + kEY[i], g.ny);
    s[i * g.plane + (long long)y * g.pitch + g.off + xx] =
        store_f64<T, SHIFT>(f[((long long)i * g.ny + sy) * g.nx + sx], i);
}

// f_i(x) = S_i(x - e_i) into a canonical FP64 array [9][ny][nx].
template <class T, bool SHIFT> __global__ void get_f_kernel(const T* __restrict__ s, Geom g, double* __restrict__ f)
{
    const RowIdx ri = row_idx(g, g.nx);
    if (!ri.ok) return;
    const int i = ri.i, y = ri.y, xx = ri.col;
    const int sy = wrapy(y - kEY[i], g.ny);
    f[((long long)i * g.ny + y) * g.nx + xx] =
        load_f64<T, SHIFT>(s[i * g.plane + (long long)sy * g.pitch + g.off + xx - kEX[i]], i);
}

// Moments (Eq. 3) of f(x, t) in FP64, optional fields, and per-block
// partial sums of (rho - 1, j_x, j_y) for the conservation totals.
constexpr int kRedThreads = 256;

template <class T, bool SHIFT>
__global__ __launch_bounds__(kRedThreads) void moments_kernel(const T* __restrict__ s, Geom g, double* __restrict__ rho,
                                                              double* __restrict__ ux, double* __restrict__ uy,
                                                              double* __restrict__ partials)
{
    __shared__ double red[3][kRedThreads];
    const long long n = (long long)g.nx * g.ny;
    const long long q = (long long)blockIdx.x * kRedThreads + threadIdx.x;
    double dr = 0.0, jx = 0.0, jy = 0.0;
    if (q < n) {
        const int y = (int)(q / g.nx), x = (int)(q - (long long)y * g.nx);
        // Shifted forms store g_i = f_i - w_i; since sum_i w_i e_i = 0 the
        // momentum is sum_i g_i e_i as well, and rho = 1 + sum_i g_i.
        double vsum = 0.0;
        for (int i = 0; i < 9; ++i) {
            const int sy = wrapy(y - kEY[i], g.ny);
            const double v = (double)s[i * g.plane + (long long)sy * g.pitch + g.off + x - kEX[i]];
            vsum += v;
            jx += v * kEX[i];
            jy += v * kEY[i];
        }
        const double r = SHIFT ? 1.0 + vsum : vsum;
        dr = SHIFT ? vsum : vsum - 1.0;
        if (rho) rho[q] = r;
        if (ux) ux[q] = jx / r;
        if (uy) uy[q] = jy / r;
    }
    red[0][threadIdx.x] = dr;
    red[1][threadIdx.x] = jx;
    red[2][threadIdx.x] = jy;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) partials[(long long)blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Fixed-order reduction of nparts partial triples; out = {N + sum drho, sum jx, sum jy}.
__global__ __launch_bounds__(kRedThreads) void reduce_partials_kernel(const double* __restrict__ partials, int nparts,
                                                                      double nsites, double* __restrict__ out)
{
    __shared__ double red[3][kRedThreads];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nparts; p += kRedThreads)
        for (int c = 0; c < 3; ++c) acc[c] += partials[(long long)p * 3 + c];
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = nsites + red[0][0];
        out[1] = red[1][0];
        out[2] = red[2][0];
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers.

template <class T, bool SHIFT, int VX, int NW> static hipError_t launch_step_t(const StepTile& t, hipStream_t st)
{
    const int ntiles = t.nstrips * t.nchunks;
    const int grid = (ntiles + 7) / 8 * 8;
    hipLaunchKernelGGL((step_kernel<T, SHIFT, VX, NW>), dim3(grid), dim3(64 * NW), 0, st, t, ntiles);
    return hipGetLastError();
}

template <class T, bool SHIFT, int VX> static hipError_t launch_nw(int nw, const StepTile& t, hipStream_t st)
{
    switch (nw) {
    case 1: return launch_step_t<T, SHIFT, VX, 1>(t, st);
    case 2: return launch_step_t<T, SHIFT, VX, 2>(t, st);
    case 4: return launch_step_t<T, SHIFT, VX, 4>(t, st);
    default: return hipErrorInvalidValue;
    }
}

bool step_shape_supported(int dtype, int vx, int nw)
{
    if (nw != 1 && nw != 2 && nw != 4) return false;
    switch (dtype) {
    case 0: return vx == 1 || vx == 2;
    case 1:
    case 2: return vx == 1 || vx == 2 || vx == 4;
    case 3: return vx == 2 || vx == 4 || vx == 8;
    default: return false;
    }
}

hipError_t launch_step(int dtype, int vx, int nw, const StepTile& t, hipStream_t st)
{
    if (!step_shape_supported(dtype, vx, nw)) return hipErrorInvalidValue;
    switch (dtype) {
    case 0:
        return vx == 1 ? launch_nw<double, false, 1>(nw, t, st) : launch_nw<double, false, 2>(nw, t, st);
    case 1:
        return vx == 1 ? launch_nw<float, false, 1>(nw, t, st)
                       : (vx == 2 ? launch_nw<float, false, 2>(nw, t, st) : launch_nw<float, false, 4>(nw, t, st));
    case 2:
        return vx == 1 ? launch_nw<float, true, 1>(nw, t, st)
                       : (vx == 2 ? launch_nw<float, true, 2>(nw, t, st) : launch_nw<float, true, 4>(nw, t, st));
    case 3:
        return vx == 2 ? launch_nw<_Float16, true, 2>(nw, t, st)
                       : (vx == 4 ? launch_nw<_Float16, true, 4>(nw, t, st) : launch_nw<_Float16, true, 8>(nw, t, st));
    }
    return hipErrorInvalidValue;
}

static dim3 plane_rows_grid(const Geom& g, int extra)
{
    const long long n = 9LL * g.ny * (g.nx + extra);
    return dim3((unsigned)((n + 255) / 256));
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
                       hipStream_t st)
{
    LBM_DISPATCH(dtype, {
        hipLaunchKernelGGL((init_kernel<T, S>), plane_rows_grid(g, 2), dim3(256), 0, st, (T*)s, g, rho, ux, uy);
        return hipGetLastError();
    })
}

hipError_t launch_set_f(int dtype, void* s, const Geom& g, const double* f, hipStream_t st)
{
    LBM_DISPATCH(dtype, {
        hipLaunchKernelGGL((set_f_kernel<T, S>), plane_rows_grid(g, 2), dim3(256), 0, st, (T*)s, g, f);
        return hipGetLastError();
    })
}

hipError_t launch_get_f(int dtype, const void* s, const Geom& g, double* f, hipStream_t st)
{
    LBM_DISPATCH(dtype, {
        hipLaunchKernelGGL((get_f_kernel<T, S>), plane_rows_grid(g, 0), dim3(256), 0, st, (const T*)s, g, f);
        return hipGetLastError();
    })
}

int moments_blocks(const Geom& g)
{
    const long long n = (long long)g.nx * g.ny;
    return (int)((n + kRedThreads - 1) / kRedThreads);
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
