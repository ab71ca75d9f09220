// internal.h -- types shared by the HIP kernels and the host runtime of liblbm.
//
// Storage ("pull" form). For every link i the device keeps one plane
// S_i[y][x] holding the post-collision value f*_i(x, y) of the previous step,
// i.e. the value that streams to x + e_i (Eq. 5, left-hand side). A step
// gathers f_i(x, t) = S_i(x - e_i), relaxes it (Eq. 5, right-hand side) and
// writes S'_i(x) aligned into the other buffer (A/B).
//
// Layout: element (x, y) of plane i sits at
//   i * ps + y * rs + off + x,   x in [0, nx)
// `off` is one 128-byte line, so x = 0 is line-aligned; the row is padded
// on both sides (the +-1-shifted windows of the gather read a little past
// the row ends and replace those elements by the periodic image, see
// gather_raw). Two layouts are supported:
// plane-major (ps = plane size, rs = pitch) and row-interleaved (ps = pitch,
// rs = 9 * pitch: the nine plane rows of a lattice row are contiguous).
// Rows wrap in y by index.
#pragma once

#include <stdint.h>

namespace lbm {

constexpr int kMaxVX = 8;

struct Geom {
    int nx, ny;
    int off;          // element offset of column 0 within a row
    int pitch;        // elements per row of one plane
    long long rs;     // elements between rows y and y + 1 of a plane
    long long ps;     // elements between planes i and i + 1
};

// Collision / source coefficients of Eq. 5 in the delta form used by the
// kernels (d_i = f_i - w_i):
//   d*_0 = om1 d_0 + wo0 A
//   d*_i = om1 d_i + P + Q,  d*_opp = om1 d_opp + P - Q        (pairs)
// with om = 1/tau, om1 = 1 - om, wo_k = om w_k, and as_k = 3 w_k alpha / 2:
// the source term 3 w_k alpha (e_i . grad rho) is applied to the undivided
// central differences rho(x + 1) - rho(x - 1), so the 1/2 of the central
// difference sits in the coefficient (an exact power-of-two scaling).
// e1, e0 shift the equilibrium for the altered-equilibrium model (0 for the
// paper's model): the moving pairs relax towards A + rho e1 in place of A,
// the rest population towards A + rho e0. The FP32-compute kernels take the
// same values rounded once to FP32.
struct Coef {
    double om1, wo0, wo1, wo2, as1, as2, e1, e0;
    float om1f, wo0f, wo1f, wo2f, as1f, as2f, e1f, e0f;
};

// One lattice as seen by a step launch.
struct StepTile {
    const void* src;
    void* dst;
    Geom g;
    Coef c;
    int h;        // rows per workgroup
    int nstrips;  // column strip groups (one per workgroup)
    int nchunks;  // row chunks
    int rowband;  // tile order: 1 = strip groups of a chunk first
    int xcd_chunk;  // vertical-stack tile order over the 8 XCDs (see xcd_tile in step.h)
    // Per-site source coefficients (a c2 field): field[y * fpitch + x] =
    // as1 at site (x, y) in compute precision (as2 = as1 / 4); nullptr for
    // the uniform coefficients of c.
    const void* field;
    int fpitch;
};

// A dispatch's work-item count is 32-bit: launchers refuse a grid that
// would exceed it (hipErrorInvalidConfiguration) rather than have it cut.
inline bool grid_fits(long long blocks, int threads) { return blocks * threads <= 0xffffffffLL; }

// The source coefficient of the axis links, as1 = 3 w_1 alpha / 2 with
// alpha = 1/3 - c2 (Eq. 8; the diagonal links take as2 = as1 / 4, exactly,
// since w_2 = w_1 / 4). One definition for the uniform coefficients and the
// per-site field, so that a uniform field gives the same bits.
__host__ __device__ inline double source_as1(double c2)
{
    const double alpha = 1.0 / 3.0 - c2;
    return 1.5 * (1.0 / 9.0) * alpha;
}

// One lattice of a batched launch (device array, read by every workgroup).
// tile.src holds the buffer of even times and tile.dst the buffer of odd
// times: at step s of the call the lattice is at time t0 + s, reads buffer
// (t0 + s) & 1 and writes the other. Lattices with s >= nsteps sit out.
// The batch's work is cut into items of up to `per_item` consecutive tiles
// of one lattice; item i belongs to lattice item_lat[i] (a device array),
// and the lattice's items are item_begin .. item_begin + nitems - 1.
struct BatchLat {
    StepTile tile;
    long long t0;    // lattice time when the call starts
    int nsteps;      // steps this lattice takes in the call
    int item_begin;  // first batch item of this lattice
    int ntiles;      // tiles of this lattice (tile.nstrips * tile.nchunks)
    int per_item;    // tiles per item
};

}  // namespace lbm
