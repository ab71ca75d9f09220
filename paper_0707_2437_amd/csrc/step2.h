// step2.h -- tile geometry of the two-step vertical-stack kernel
// (step2.hip), shared by its launcher and the host runtime.
#pragma once

namespace lbm {

// A two-step tile advances a block of sites by two steps of Eq. 5 in one
// pass over memory. Each lane gathers its own vx columns and takes its
// x-neighbours' densities from its neighbour lanes, so the first step has
// no result at the outermost column on either side of a 64-lane strip. The
// second step at a column needs first-step results up to two columns away
// (its gather and its neighbours' densities), so a strip writes the columns
// from the fourth to the fourth last: ceil(3 / vx) lanes at each side only
// supply the first step. (For vx = 2, a strip writes 120 columns, which
// also keeps the strips' boundaries on 32-byte sectors of FP32 rows.)
constexpr int step2_halo_lanes(int vx) { return (3 + vx - 1) / vx; }
constexpr int step2_cols(int vx) { return (64 - 2 * step2_halo_lanes(vx)) * vx; }
// Vertically the second step's density gradient needs its gathers one row
// above and below, those need first-step results one more row out, and
// those need first-step densities one more row out: a tile of nw rows (one
// per wave, or two per wave for nw = 32) writes nw - 6 rows.
constexpr int step2_rows(int nw) { return nw - 6; }

}  // namespace lbm
