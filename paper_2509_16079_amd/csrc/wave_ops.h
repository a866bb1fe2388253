// wave_ops.h -- cross-lane FP64 helpers for 64-lane gfx950 wavefronts
// (DPP moves and readlanes: no LDS traffic). Callers keep every lane of the
// wave active where they call these.
#pragma once

#include <hip/hip_runtime.h>

namespace vpm {

// Value of v in lane j (uniform j) for every lane: two readlanes, no LDS.
__device__ inline double bcast(double v, int j) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(static_cast<unsigned>(u), j);
  const unsigned hi = __builtin_amdgcn_readlane(static_cast<unsigned>(u >> 32), j);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// v from another lane of the same 16-lane row, by DPP control CTRL.
template <int CTRL>
__device__ inline double dpp(double v) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(static_cast<long long>(
      (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo)));
}

// v from another lane by DPP control CTRL into the 16-lane rows set in ROWS;
// the other rows get 0.
template <int CTRL, int ROWS>
__device__ inline double dpp_rows(double v) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(static_cast<long long>(
      (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo)));
}

// Sum of v over the 64 lanes (all active), in every lane, in a fixed order:
// pairs, quads, then 8- and 16-lane rows by DPP (no LDS), then the four row
// sums r0..r3 as (r2 + r3) + (r0 + r1): row_bcast:15 adds row 0's sum to
// row 1 and row 2's to row 3, row_bcast:31 adds lane 31 (r0 + r1) to row 3,
// and lane 63's total is broadcast.
__device__ inline double wave_sum(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x124>(v);  // row_ror:4
  v += dpp<0x128>(v);  // row_ror:8
  v += dpp_rows<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_rows<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return bcast(v, 63);
}

}  // namespace vpm
