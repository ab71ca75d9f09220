// step2.h -- tile geometry of the two-step vertical-stack kernel
// (step2.hip), shared by its launcher and the host runtime.
#pragma once

namespace lbm {

// A two-step tile advances a block of sites by two steps of Eq. 5 in one
// pass over memory. The second step at a site needs the first step's
// results at the sites up to two columns away (its gather and the densities
// of its x-neighbours), and those need the stored values up to one more
// column away, which each lane's window already loads. So a strip of 64
// lanes writes the columns of its inner lanes and leaves ceil(2 / vx) lanes
// at each side to supply only the first step.
constexpr int step2_halo_lanes(int vx) { return (2 + vx - 1) / vx; }
constexpr int step2_cols(int vx) { return (64 - 2 * step2_halo_lanes(vx)) * vx; }
// Vertically the second step's density gradient needs its gathers one row
// above and below, those need first-step results one more row out, and
// those need first-step densities one more row out: a workgroup of nw waves
// (one row each) writes nw - 6 rows.
constexpr int step2_rows(int nw) { return nw - 6; }

}  // namespace lbm
