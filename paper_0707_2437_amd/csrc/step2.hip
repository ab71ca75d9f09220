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
//   1. the waves gather their rows' own columns from memory (Eq. 5,
//      left-hand side: plane i from column x - e_ix of row y - e_iy) and
//      publish the densities in LDS, one row per wave;
//   2. waves 1 .. NW-2 relax (first step) into LDS, rounded to the storage
//      type: the values a single step would store; the density gradient
//      takes the x-neighbours from the wave's own LDS row and the
//      y-neighbours from the rows above and below;
//   3. waves 2 .. NW-3 gather from those and publish the new densities;
//   4. waves 3 .. NW-4, inner lanes only, relax (second step) and write.
// Every site's arithmetic is the single-step code of step.h (the same drho
// and collide functions, on the same inputs), so a two-step pass gives the
// bits of two single steps. FP16 storage takes the same code with each
// value converted to FP32 where it is used: the single-step FP16 kernel
// reads its halves as operands of mixed-precision FMAs, which convert them
// exactly and round once, the same bits. Its rows' ghost columns (see
// GhostCols in step.h) are written with the second step's results.
#include <hip/hip_runtime.h>

#include "grid_sync.h"
#include "internal.h"
#include "step.h"
#include "step2.h"

namespace lbm {

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Own-column gather of a lane whose sources may wrap: f_i at column x + j
// is S_i at column x + j - e_ix, taken mod nx; rb are the source rows of
// the nine planes (row_bases in step.h). The columns are x - 1 + k with
// k = j + 1 - e_ix in [0, VX + 1]: one remainder per lane, x0 = (x - 1) mod
// nx, then x0 + k <= nx + VX < 3 nx, so at most two subtractions of nx.
template <class T, int VX>
__device__ __forceinline__ void gather_own_wrapped(const char* const (&rb)[9], const Geom& g, int x,
                                                   T (&v)[9][VX])
{
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static_assert(VX <= 5, "two subtractions of nx suffice for nx >= 3");
    constexpr unsigned es = sizeof(T);
    const int x0 = wrap_mod(x - 1, g.nx);
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            int s = x0 + (j + 1 - ex[i]);
            s = s >= g.nx ? s - g.nx : s;
            s = s >= g.nx ? s - g.nx : s;
            v[i][j] = ld_g<T>(rb[i] + (size_t)((unsigned)(s + 2) * es));
        }
}

// The per-site source coefficients (a c2 field, array of row pitch
// a.fpitch in compute precision) of the lane's columns of row r in
// [0, ny); columns outside the lattice are taken mod nx as in
// gather_own_wrapped. The field does not change with time, so one load
// serves both steps.
template <class C, int VX>
__device__ __forceinline__ void field_own(const StepTile& a, int r, int x, bool edge, C (&af)[VX])
{
    const char* row = (const char*)a.field + (size_t)r * a.fpitch * sizeof(C);
    if (edge) {
        const int x0 = wrap_mod(x, a.g.nx);
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            const int s = x0 + j >= a.g.nx ? x0 + j - a.g.nx : x0 + j;
            af[j] = ld_g<C>(row + (size_t)((unsigned)s * sizeof(C)));
        }
    } else {
        const Pack<C, VX> p = ld_vec<C, VX, 4>(row, (unsigned)x * (unsigned)sizeof(C));
#pragma unroll
        for (int j = 0; j < VX; ++j) af[j] = p.v[j];
    }
}

// Base pointers of the nine planes at column c0 of row r (in [0, ny)) of
// buffer buf; with SHIFT_ROWS plane i is taken at row r - e_iy (wrapped).
// The planes are stepped through with 64-bit additions (the planes of the
// plane-major layout may span more than 4 GB together); row offsets are
// 32-bit products (a plane, and a row-interleaved buffer, spans less than
// 4 GB: offsets_fit on the host).
template <class T, bool SHIFT_ROWS>
__device__ __forceinline__ void plane_rows(const void* buf, const Geom& g, int c0, int r, const char* (&p)[9])
{
    constexpr unsigned es = sizeof(T);
    constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const unsigned rsb = (unsigned)g.rs * es;
    const unsigned long long psb = (unsigned long long)g.ps * es;
    const unsigned o0 = (unsigned)r * rsb;
    const unsigned om = SHIFT_ROWS ? (unsigned)(r == 0 ? g.ny - 1 : r - 1) * rsb : o0;
    const unsigned op = SHIFT_ROWS ? (unsigned)(r == g.ny - 1 ? 0 : r + 1) * rsb : o0;
    const char* q = (const char*)buf + (long long)(g.off + c0) * (long long)es;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        p[i] = q + (ey[i] > 0 ? om : (ey[i] < 0 ? op : o0));
        q += psb;
    }
}

// LDS of a two-step tile: the densities (one row per wave) and the first
// step's results of waves 1 .. NW - 2, in rows of the lanes' columns plus
// one column on each side.
template <class T, int VX, int NW> struct Step2Lds {
    static constexpr int LW = 64 * VX + 2;
    typename CompT<T>::type rho[NW][LW];
    T fs[NW - 2][9][LW];
};

// One two-step tile: strip `strip`, row group `grp` of lattice a, reading
// src and writing dst. single: take one step only (the group's rows and
// the strip's columns as for two steps, phases 1 and 4 of the header with
// the relaxed rows written; the lone last step of an odd step count in the
// batched form). FIELD: the lattice has a c2 field. RC: centre the
// arithmetic on the lattice model's state at rest (see Centre in step.h).
// Every wave of the workgroup must call it (it holds workgroup barriers);
// the caller places a barrier between two calls that reuse lds.
// KIND: a distinct instantiation per kernel that uses the tile (measured:
// sharing one instantiation between the grouped and persistent batched
// kernels made the compiler spill registers in the grouped one).
template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD, bool RC, int KIND = 0>
__device__ __forceinline__ void step2_tile(const StepTile& a, const void* src, void* dst, int strip, int grp,
                                           bool single, Step2Lds<T, VX, NW>& lds)
{
    using C = typename CompT<T>::type;
    using K = KeepT<T, C>;
    constexpr int HL = step2_halo_lanes(VX);
    constexpr int W2 = step2_cols(VX);
    constexpr int R2 = step2_rows(NW);
    static_assert(R2 >= 1, "a two-step tile needs at least 7 waves");
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr unsigned es = sizeof(T);
    auto& rho = lds.rho;
    auto& fs = lds.fs;
    // LDS column c -> slot: with two columns per lane, even and odd columns
    // in the two halves of a row, so that lanes touch consecutive slots
    constexpr int HW = Step2Lds<T, VX, NW>::LW / 2;
    auto li = [](int c) { return VX == 2 ? (c & 1) * HW + (c >> 1) : c; };

    const Geom g = a.g;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int y0 = grp * R2;
    const int nrows = min(R2, g.ny - y0);
    const int y = y0 - 3 + wave;
    const int xs = strip * W2;
    const int x = xs + (lane - HL) * VX;
    // sources of the strip: columns x - 1 .. x + VX of every lane
    const bool edge = xs - HL * VX - 1 < 0 || xs + (64 - HL) * VX + 1 > g.nx;
    const CoefC<C> k = coef_c<C>(a.c);
    const Centre<C> cn = centre_c<C, RC>(a.c);
    const int col = lane * VX + 1;  // LDS column of the lane's first column
    const int nv = min(VX, g.nx - x);
    // the rows and lanes the tile writes
    const bool out = wave >= 3 && wave <= nrows + 2 && lane >= HL && lane < 64 - HL && nv > 0;

    K d[9][VX];
    C w[VX];
    C af[VX] = {};  // per-site source coefficients (FIELD)
    // densities and x differences of the lane's columns from a row of LDS
    auto relax = [&](const C* rrow, const C* rup, const C* rdn, C (&o)[VX][9]) {
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            const C left = j == 0 ? rrow[li(col - 1)] : w[j - 1];
            const C right = j == VX - 1 ? rrow[li(col + VX)] : w[j + 1];
            // undivided central differences at time t (Sec. 4)
            const C gx = right - left;
            const C gy = rup[li(col + j)] - rdn[li(col + j)];
            collide<T, SHIFT, C, VX, RC>(d, j, w[j], gx, gy, site_coef<FIELD>(k, af[j]), cn, o[j]);
        }
    };
    auto write = [&](const C (&o)[VX][9]) {
        Pack<T, VX> pk[9];
#pragma unroll
        for (int j = 0; j < VX; ++j)
#pragma unroll
            for (int i = 0; i < 9; ++i) pk[i].v[j] = from_d<T, SHIFT, C>(o[j][i], i, cn);
        char* dbase[9];
        if constexpr (VX == 1) {
            // the row's plane bases as for the loads (measured faster with one
            // column per lane, slower with two)
            const char* rows[9];
            plane_rows<T, false>(dst, g, 0, y, rows);
#pragma unroll
            for (int i = 0; i < 9; ++i) dbase[i] = const_cast<char*>(rows[i]);
            write_row<T, VX, NTS>(dbase, g, 0, x, nv, pk);  // the row is in dbase
        } else {
            dst_bases<T>(dst, g, dbase);
            write_row<T, VX, NTS>(dbase, g, y, x, nv, pk);
        }
    };
    // 1. Gather the own columns from memory: rows 0 .. nrows + 5 for two
    // steps, 2 .. nrows + 3 for one; the other waves idle.
    const bool load = single ? (wave >= 2 && wave <= nrows + 3) : (wave <= nrows + 5);
    if (load) {
        // y in [-3, ny + 2] and ny >= 3: one wrap
        const int yw = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
        const char* rb[9];
        plane_rows<T, true>(src, g, -2, yw, rb);
        if constexpr (FIELD)
            if (single ? (wave >= 3 && wave <= nrows + 2) : (wave >= 1 && wave <= nrows + 4))
                field_own<C, VX>(a, yw, x, edge, af);
        T raw[9][VX];
        if (edge) {
            gather_own_wrapped<T, VX>(rb, g, x, raw);
        } else {
            constexpr int A = es < 4 ? (int)es : 4;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const Pack<T, VX> p = ld_vec<T, VX, A>(rb[i], (unsigned)(x - ex[i] + 2) * es);
#pragma unroll
                for (int j = 0; j < VX; ++j) raw[i][j] = p.v[j];
            }
        }
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < VX; ++j) d[i][j] = keep_of<T, SHIFT, C>(raw[i][j], i, cn);
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            w[j] = drho_of<T, SHIFT, C, VX>(d, j, cn);
            rho[wave][li(col + j)] = w[j];
        }
    }
    __syncthreads();
    if (single) {  // one step: relax and write the group's rows
        if (out) {
            C o[VX][9];
            relax(rho[wave], rho[wave + 1], rho[wave - 1], o);
            write(o);
        }
        return;
    }
    // 2. First step, every lane, into LDS.
    if (wave >= 1 && wave <= min(nrows + 4, NW - 2)) {
        C o[VX][9];
        relax(rho[wave], rho[wave + 1], rho[wave - 1], o);
#pragma unroll
        for (int j = 0; j < VX; ++j)
#pragma unroll
            for (int i = 0; i < 9; ++i) fs[wave - 1][i][li(col + j)] = from_d<T, SHIFT, C>(o[j][i], i, cn);
    }
    __syncthreads();
    // 3. Second gather, from LDS: f_i at column c of row y is the first
    // step's S_i at column c - e_ix of row y - e_iy. Lanes next to the strip
    // edge read LDS columns that nothing wrote; their results are never written.
    if (wave >= 2 && wave <= min(nrows + 3, NW - 3)) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < VX; ++j)
                d[i][j] = keep_of<T, SHIFT, C>(fs[wave - ey[i] - 1][i][li(col + j - ex[i])], i, cn);
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            w[j] = drho_of<T, SHIFT, C, VX>(d, j, cn);
            rho[wave][li(col + j)] = w[j];
        }
    }
    __syncthreads();
    // 4. Second step: the group's rows, inner lanes, columns inside the lattice.
    if (out) {
        C o[VX][9];
        relax(rho[wave], rho[wave + 1], rho[wave - 1], o);
        write(o);
    }
}

// The single-lattice kernel's tile: as step2_tile below, for tiles of NW
// rows on step2_waves(NW) waves (two rows per wave for 32-row tiles). The
// batched kernels keep the one-row form: this one's registers spill there,
// under their 8-waves-per-SIMD target.
//
// One two-step tile (NW rows, step2_waves(NW) waves): strip `strip`, row
// group `grp` of lattice a, reading
// src and writing dst. single: take one step only (the group's rows and
// the strip's columns as for two steps, phases 1 and 4 of the header with
// the relaxed rows written; the lone last step of an odd step count in the
// batched form). FIELD: the lattice has a c2 field. RC: centre the
// arithmetic on the lattice model's state at rest (see Centre in step.h).
// Every wave of the workgroup must call it (it holds workgroup barriers);
// the caller places a barrier between two calls that reuse lds.
// KIND: a distinct instantiation per kernel that uses the tile (measured:
// sharing one instantiation between the grouped and persistent batched
// kernels made the compiler spill registers in the grouped one).
// Waves of a two-step tile of NW rows: one row per wave up to 16 waves (the
// most a workgroup holds), two rows per wave for 32-row tiles (one column
// per lane and 4-byte or smaller storage, whose LDS still lets two
// workgroups share a CU). Wave w then holds tile rows w and w + 16, and
// every phase runs over both.
constexpr int step2_waves(int nw) { return nw > 16 ? 16 : nw; }

template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD, bool RC>
__device__ __forceinline__ void step2_tile_rows(const StepTile& a, const void* src, void* dst, int strip, int grp,
                                           bool single, Step2Lds<T, VX, NW>& lds)
{
    using C = typename CompT<T>::type;
    using K = KeepT<T, C>;
    constexpr int NWAVES = step2_waves(NW);
    constexpr int RPW = NW / NWAVES;  // rows per wave
    static_assert(RPW * NWAVES == NW, "rows a multiple of the waves");
    constexpr int HL = step2_halo_lanes(VX);
    constexpr int W2 = step2_cols(VX);
    constexpr int R2 = step2_rows(NW);
    static_assert(R2 >= 1, "a two-step tile needs at least 7 rows");
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr unsigned es = sizeof(T);
    auto& rho = lds.rho;
    auto& fs = lds.fs;
    constexpr int HW = Step2Lds<T, VX, NW>::LW / 2;
    auto li = [](int c) { return VX == 2 ? (c & 1) * HW + (c >> 1) : c; };

    const Geom g = a.g;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int y0 = grp * R2;
    const int nrows = min(R2, g.ny - y0);
    const int xs = strip * W2;
    const int x = xs + (lane - HL) * VX;
    const bool edge = xs - HL * VX - 1 < 0 || xs + (64 - HL) * VX + 1 > g.nx;
    const CoefC<C> k = coef_c<C>(a.c);
    const Centre<C> cn = centre_c<C, RC>(a.c);
    const int col = lane * VX + 1;
    const int nv = min(VX, g.nx - x);
    const bool lane_out = lane >= HL && lane < 64 - HL && nv > 0;

    K d[RPW][9][VX];
    C w[RPW][VX];
    C af[RPW][VX] = {};
    auto relax = [&](int q, int r, C (&o)[VX][9]) {
        const C* rrow = rho[r];
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            const C left = j == 0 ? rrow[li(col - 1)] : w[q][j - 1];
            const C right = j == VX - 1 ? rrow[li(col + VX)] : w[q][j + 1];
            const C gx = right - left;
            const C gy = rho[r + 1][li(col + j)] - rho[r - 1][li(col + j)];
            collide<T, SHIFT, C, VX, RC>(d[q], j, w[q][j], gx, gy, site_coef<FIELD>(k, af[q][j]), cn, o[j]);
        }
    };
    auto write = [&](int r, const C (&o)[VX][9]) {
        const int y = y0 - 3 + r;
        Pack<T, VX> pk[9];
#pragma unroll
        for (int j = 0; j < VX; ++j)
#pragma unroll
            for (int i = 0; i < 9; ++i) pk[i].v[j] = from_d<T, SHIFT, C>(o[j][i], i, cn);
        char* dbase[9];
        if constexpr (VX == 1) {
            const char* rows[9];
            plane_rows<T, false>(dst, g, 0, y, rows);
#pragma unroll
            for (int i = 0; i < 9; ++i) dbase[i] = const_cast<char*>(rows[i]);
            write_row<T, VX, NTS>(dbase, g, 0, x, nv, pk);
        } else {
            dst_bases<T>(dst, g, dbase);
            write_row<T, VX, NTS>(dbase, g, y, x, nv, pk);
        }
    };
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int r = wave + q * NWAVES;  // the tile row, at lattice row y0 - 3 + r
        const bool load = single ? (r >= 2 && r <= nrows + 3) : (r <= nrows + 5);
        if (load) {
            const int y = y0 - 3 + r;
            const int yw = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
            const char* rb[9];
            plane_rows<T, true>(src, g, -2, yw, rb);
            if constexpr (FIELD)
                if (single ? (r >= 3 && r <= nrows + 2) : (r >= 1 && r <= nrows + 4))
                    field_own<C, VX>(a, yw, x, edge, af[q]);
            T raw[9][VX];
            if (edge) {
                gather_own_wrapped<T, VX>(rb, g, x, raw);
            } else {
                constexpr int A = es < 4 ? (int)es : 4;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const Pack<T, VX> p = ld_vec<T, VX, A>(rb[i], (unsigned)(x - ex[i] + 2) * es);
#pragma unroll
                    for (int j = 0; j < VX; ++j) raw[i][j] = p.v[j];
                }
            }
#pragma unroll
            for (int i = 0; i < 9; ++i)
#pragma unroll
                for (int j = 0; j < VX; ++j) d[q][i][j] = keep_of<T, SHIFT, C>(raw[i][j], i, cn);
#pragma unroll
            for (int j = 0; j < VX; ++j) {
                w[q][j] = drho_of<T, SHIFT, C, VX>(d[q], j, cn);
                rho[r][li(col + j)] = w[q][j];
            }
        }
    }
    __syncthreads();
    if (single) {
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int r = wave + q * NWAVES;
            if (r >= 3 && r <= nrows + 2 && lane_out) {
                C o[VX][9];
                relax(q, r, o);
                write(r, o);
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int r = wave + q * NWAVES;
        if (r >= 1 && r <= min(nrows + 4, NW - 2)) {
            C o[VX][9];
            relax(q, r, o);
#pragma unroll
            for (int j = 0; j < VX; ++j)
#pragma unroll
                for (int i = 0; i < 9; ++i) fs[r - 1][i][li(col + j)] = from_d<T, SHIFT, C>(o[j][i], i, cn);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int r = wave + q * NWAVES;
        if (r >= 2 && r <= min(nrows + 3, NW - 3)) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
#pragma unroll
                for (int j = 0; j < VX; ++j)
                    d[q][i][j] = keep_of<T, SHIFT, C>(fs[r - ey[i] - 1][i][li(col + j - ex[i])], i, cn);
#pragma unroll
            for (int j = 0; j < VX; ++j) {
                w[q][j] = drho_of<T, SHIFT, C, VX>(d[q], j, cn);
                rho[r][li(col + j)] = w[q][j];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int r = wave + q * NWAVES;
        if (r >= 3 && r <= nrows + 2 && lane_out) {
            C o[VX][9];
            relax(q, r, o);
            write(r, o);
        }
    }
}

// FIELD: a lattice with a c2 field (per-site source coefficients).
template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD>
__global__ __launch_bounds__(64 * step2_waves(NW)) void step2_vstack_kernel(StepTile a, int ntiles)
{
    __shared__ Step2Lds<T, VX, NW> lds;
    const int t = xcd_tile(blockIdx.x, gridDim.x, a.xcd_chunk);
    if (t >= ntiles) return;
    step2_tile_rows<T, SHIFT, VX, NW, NTS, FIELD, ModelCentred<typename CompT<T>::type>::value>(
        a, a.src, a.dst, t % a.nstrips, t / a.nstrips, false, lds);
}

// Batched form: pass p (steps 2p and 2p + 1) of every lattice of a batch
// (BatchLat in internal.h; one workgroup per item, items dealt to the XCDs
// in chunks of ch, see xcd_tile). A lattice's descriptor carries as t0 its
// buffer time: the state at the start of the call is in buffer t0 & 1
// (tile.src for even, tile.dst for odd), and every pass moves it to the
// other buffer. A lattice with nsteps <= 2p sits out; one with nsteps =
// 2p + 1 takes its last step alone. Pools step the paper's model, centred
// on the weights (as the single-step batched kernels).
// The 16-wave shapes whose LDS lets two workgroups share a CU are compiled
// for 8 waves per SIMD: left to itself the compiler spends more scalar
// registers than that allows.
template <class T, bool SHIFT, int VX, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 16 && sizeof(T) * VX <= 8 ? 8 : 1, 8))) void batch_step2_kernel(const BatchLat* __restrict__ lats,
                                                              const int* __restrict__ item_lat, int nitems, int p,
                                                              int ch)
{
    __shared__ Step2Lds<T, VX, NW> lds;
    const int i = xcd_tile(blockIdx.x, gridDim.x, ch);
    if (i >= nitems) return;
    const BatchLat& L = lats[item_lat[i]];
    if (2 * p >= L.nsteps) return;
    const bool single = 2 * p + 1 == L.nsteps;
    const bool odd = ((L.t0 + p) & 1) != 0;
    const void* src = odd ? L.tile.dst : L.tile.src;
    void* dst = odd ? const_cast<void*>(L.tile.src) : L.tile.dst;
    const int t0 = (i - L.item_begin) * L.per_item;
    const int t1 = min(t0 + L.per_item, L.ntiles);
    for (int t = t0; t < t1; ++t) {
        if (t > t0) __syncthreads();  // lds of the previous tile is still being read
        step2_tile<T, SHIFT, VX, NW, NTS, false, false>(L.tile, src, dst, t % L.tile.nstrips, t / L.tile.nstrips,
                                                        single, lds);
    }
}

// Persistent form: all npasses passes of a batch in one launch whose G
// member workgroups (join_members in grid_sync.h) meet at a grid barrier
// between passes, since pass p + 1 reads what pass p wrote. Work is taken
// dynamically as in the single-step persistent kernel (batch.hip): one
// counter per part and pass (two passes' sets alternate; the barrier's last
// arriver zeroes the next pass's set), a member takes its part's next item
// with one atomic add, so a pass ends when its work does. Each item is run
// as in batch_step2_kernel.
template <class T, bool SHIFT, int VX, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 16 && sizeof(T) * VX <= 8 ? 8 : 1, 8))) void batch_persistent2_kernel(
    const BatchLat* __restrict__ lats, const int* __restrict__ item_lat, int nitems, int npasses, int ch,
    unsigned* bar, unsigned long long wait_ticks, unsigned long long grace_ticks)
{
    __shared__ Step2Lds<T, VX, NW> lds;
    __shared__ int next_item;
    if (stale_barrier_error(bar)) return;
    int rank = 0;
    const int G = join_members(bar, wait_ticks, grace_ticks, &rank);
    if (G == 0) return;
    const bool by_xcd = G == (int)gridDim.x && G % 8 == 0;
    const int nparts = by_xcd ? 8 : 1;
    const int part = by_xcd ? (int)(blockIdx.x & 7u) : 0;
    const int chunk = ch > 0 ? ch : 1;
    for (int p = 0; p < npasses; ++p) {
        unsigned* ctr = bar + kBarCtr + (p & 1) * 8 + part;
        for (;;) {
            if (threadIdx.x == 0) next_item = min(part_item((int)atomicAdd(ctr, 1u), part, nparts, chunk), nitems);
            __syncthreads();
            const int i = next_item;
            __syncthreads();  // read by every wave before the next item is written; lds free again
            if (i >= nitems) break;
            const BatchLat* L = &lats[ldc(&item_lat[i])];
            const int n = ldc(&L->nsteps);
            if (2 * p >= n) continue;  // this lattice takes fewer steps
            const bool single = 2 * p + 1 == n;
            const StepTile a = ldc(&L->tile);
            const bool odd = ((ldc(&L->t0) + p) & 1) != 0;
            const void* src = odd ? a.dst : a.src;
            void* dst = odd ? const_cast<void*>(a.src) : a.dst;
            const int per = ldc(&L->per_item);
            const int t0 = (i - ldc(&L->item_begin)) * per;
            const int t1 = min(t0 + per, ldc(&L->ntiles));
            for (int t = t0; t < t1; ++t) {
                if (t > t0) __syncthreads();  // lds of the previous tile is still being read
                step2_tile<T, SHIFT, VX, NW, NTS, false, false, 1>(a, src, dst, t % a.nstrips, t / a.nstrips,
                                                                   single, lds);
            }
        }
        if (!grid_barrier(bar, G, wait_ticks, bar + kBarCtr + ((p + 1) & 1) * 8, p + 1 < npasses ? 8 : 0)) return;
    }
}

template <class T, bool SHIFT, int VX, int NW>
static hipError_t launch2_t(bool nts, const StepTile& t, hipStream_t st)
{
    const int ntiles = t.nstrips * t.nchunks;  // strips x row groups
    const int q = t.xcd_chunk > 0 ? 8 * t.xcd_chunk : 8;
    const int grid = (ntiles + q - 1) / q * q;
    if (!grid_fits(grid, 64 * step2_waves(NW))) return hipErrorInvalidConfiguration;
    const dim3 gd(grid), bd(64 * step2_waves(NW));
    if (t.field) {
        if (nts) hipLaunchKernelGGL((step2_vstack_kernel<T, SHIFT, VX, NW, true, true>), gd, bd, 0, st, t, ntiles);
        else hipLaunchKernelGGL((step2_vstack_kernel<T, SHIFT, VX, NW, false, true>), gd, bd, 0, st, t, ntiles);
    } else {
        if (nts) hipLaunchKernelGGL((step2_vstack_kernel<T, SHIFT, VX, NW, true, false>), gd, bd, 0, st, t, ntiles);
        else hipLaunchKernelGGL((step2_vstack_kernel<T, SHIFT, VX, NW, false, false>), gd, bd, 0, st, t, ntiles);
    }
    return hipGetLastError();
}

template <class T, bool SHIFT, int VX>
static hipError_t launch2_nw(int nw, bool nts, const StepTile& t, hipStream_t st)
{
    switch (nw) {
    case 12: return launch2_t<T, SHIFT, VX, 12>(nts, t, st);
    case 16: return launch2_t<T, SHIFT, VX, 16>(nts, t, st);
    case 32:
        if constexpr (VX == 1 && sizeof(T) <= 4) return launch2_t<T, SHIFT, VX, 32>(nts, t, st);
        return hipErrorInvalidValue;
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

template <class T, bool SHIFT, int VX, int NW>
static hipError_t launch_batch2_t(bool nts, const BatchLat* lats, const int* item_lat, int nitems, int p, int ch,
                                  hipStream_t st)
{
    const int q = ch > 0 ? 8 * ch : 8;
    const int grid = (nitems + q - 1) / q * q;
    constexpr int threads = 64 * step2_waves(NW);
    if (nitems <= 0) return hipSuccess;
    if (!grid_fits(grid, threads)) return hipErrorInvalidConfiguration;
    if (nts)
        hipLaunchKernelGGL((batch_step2_kernel<T, SHIFT, VX, NW, true>), dim3(grid), dim3(threads), 0, st, lats,
                           item_lat, nitems, p, ch);
    else
        hipLaunchKernelGGL((batch_step2_kernel<T, SHIFT, VX, NW, false>), dim3(grid), dim3(threads), 0, st, lats,
                           item_lat, nitems, p, ch);
    return hipGetLastError();
}

template <class T, bool SHIFT, int VX, int NW>
static hipError_t launch_batch2_persistent_t(bool nts, const BatchLat* lats, const int* item_lat, int nitems,
                                             int npasses, int max_grid, int ch, unsigned* bar, hipStream_t st)
{
    const void* kern = nts ? (const void*)batch_persistent2_kernel<T, SHIFT, VX, NW, true>
                           : (const void*)batch_persistent2_kernel<T, SHIFT, VX, NW, false>;
    constexpr int threads = 64 * step2_waves(NW);
    int grid = 0;
    unsigned long long wait_ticks = 0, grace_ticks = 0;
    hipError_t e = persistent_setup(kern, threads, max_grid, &ch, &grid, &wait_ticks, &grace_ticks, bar, st);
    if (e != hipSuccess) return e;
    // an ordinary launch: the membership makes it correct whether or not
    // every workgroup is resident at once
    if (nts)
        hipLaunchKernelGGL((batch_persistent2_kernel<T, SHIFT, VX, NW, true>), dim3(grid), dim3(threads), 0, st,
                           lats, item_lat, nitems, npasses, ch, bar, wait_ticks, grace_ticks);
    else
        hipLaunchKernelGGL((batch_persistent2_kernel<T, SHIFT, VX, NW, false>), dim3(grid), dim3(threads), 0, st,
                           lats, item_lat, nitems, npasses, ch, bar, wait_ticks, grace_ticks);
    return hipGetLastError();
}

template <class T, bool SHIFT>
static hipError_t launch_batch2_pers_vx(int vx, int nw, bool nts, const BatchLat* lats, const int* item_lat,
                                        int nitems, int npasses, int max_grid, int ch, unsigned* bar, hipStream_t st)
{
#define LBM_P2(VXV, NWV)                                                                                          \
    if (vx == VXV && nw == NWV)                                                                                   \
        return launch_batch2_persistent_t<T, SHIFT, VXV, NWV>(nts, lats, item_lat, nitems, npasses, max_grid, ch, \
                                                              bar, st);
    LBM_P2(1, 12)
    LBM_P2(1, 16)
    LBM_P2(2, 12)
    LBM_P2(2, 16)
#undef LBM_P2
    return hipErrorInvalidValue;
}

template <class T, bool SHIFT>
static hipError_t launch_batch2_vx(int vx, int nw, bool nts, const BatchLat* lats, const int* item_lat, int nitems,
                                   int p, int ch, hipStream_t st)
{
    if (vx == 1 && nw == 12) return launch_batch2_t<T, SHIFT, 1, 12>(nts, lats, item_lat, nitems, p, ch, st);
    if (vx == 1 && nw == 16) return launch_batch2_t<T, SHIFT, 1, 16>(nts, lats, item_lat, nitems, p, ch, st);
    if (vx == 2 && nw == 12) return launch_batch2_t<T, SHIFT, 2, 12>(nts, lats, item_lat, nitems, p, ch, st);
    if (vx == 2 && nw == 16) return launch_batch2_t<T, SHIFT, 2, 16>(nts, lats, item_lat, nitems, p, ch, st);
    return hipErrorInvalidValue;
}

// dtype: 0 FP64, 1 FP32, 2 FP32-shifted, 3 FP16-shifted.
bool step2_shape_supported(int dtype, int vx, int nw)
{
    return dtype >= 0 && dtype <= 3 && (vx == 1 || vx == 2) && (nw == 12 || nw == 16 || (nw == 32 && vx == 1 && dtype != 0));
}

// flags: LBM_TILE_NT_STORE (2) selects non-temporal stores.
hipError_t launch_step2(int dtype, int vx, int nw, int flags, const StepTile& t, hipStream_t st)
{
    if (!step2_shape_supported(dtype, vx, nw)) return hipErrorInvalidValue;
    const bool nts = (flags & 2) != 0;
    switch (dtype) {
    case 0: return launch2_vx<double, false>(vx, nw, nts, t, st);
    case 1: return launch2_vx<float, false>(vx, nw, nts, t, st);
    case 2: return launch2_vx<float, true>(vx, nw, nts, t, st);
    case 3: return launch2_vx<_Float16, true>(vx, nw, nts, t, st);
    }
    return hipErrorInvalidValue;
}

// Batched form, pass p (see batch_step2_kernel); the lattices' tiles are
// those of step2_cols / step2_rows.
hipError_t launch_batch2(int dtype, int vx, int nw, bool nts, const BatchLat* lats, const int* item_lat, int nitems,
                         int p, int ch, hipStream_t st)
{
    if (!step2_shape_supported(dtype, vx, nw)) return hipErrorInvalidValue;
    switch (dtype) {
    case 0: return launch_batch2_vx<double, false>(vx, nw, nts, lats, item_lat, nitems, p, ch, st);
    case 1: return launch_batch2_vx<float, false>(vx, nw, nts, lats, item_lat, nitems, p, ch, st);
    case 2: return launch_batch2_vx<float, true>(vx, nw, nts, lats, item_lat, nitems, p, ch, st);
    case 3: return launch_batch2_vx<_Float16, true>(vx, nw, nts, lats, item_lat, nitems, p, ch, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batch2_persistent(int dtype, int vx, int nw, bool nts, const BatchLat* lats, const int* item_lat,
                                    int nitems, int npasses, int max_grid, int ch, unsigned* bar, hipStream_t st)
{
    if (!step2_shape_supported(dtype, vx, nw) || npasses < 1) return hipErrorInvalidValue;
    switch (dtype) {
    case 0: return launch_batch2_pers_vx<double, false>(vx, nw, nts, lats, item_lat, nitems, npasses, max_grid, ch, bar, st);
    case 1: return launch_batch2_pers_vx<float, false>(vx, nw, nts, lats, item_lat, nitems, npasses, max_grid, ch, bar, st);
    case 2: return launch_batch2_pers_vx<float, true>(vx, nw, nts, lats, item_lat, nitems, npasses, max_grid, ch, bar, st);
    case 3: return launch_batch2_pers_vx<_Float16, true>(vx, nw, nts, lats, item_lat, nitems, npasses, max_grid, ch, bar, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
