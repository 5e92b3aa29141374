// stencil_dev.h -- device pieces of the 7-point update (Sec. 3.1) shared by
// the stencil kernels and the fused decode / stencil / encode kernel: one cell
// update in a fixed operation order (so that every kernel gives the same bits
// for the same inputs) and one-lane wave shifts.
#pragma once
#include <hip/hip_runtime.h>

#include "oc_kernels.h"

namespace {

// One cell update in a fixed operation order, shared by every kernel here so
// that fused and single-step launches give bit-identical results.
__device__ __forceinline__ float star7_point(float c0, float cur, float xm, float xp, float ym,
                                             float yp, float zm, float zp, const oc::Star7Coef &c) {
  float r = c0 * cur;
  r = fmaf(c.cmx, xm, r);
  r = fmaf(c.cpx, xp, r);
  r = fmaf(c.cmy, ym, r);
  r = fmaf(c.cpy, yp, r);
  r = fmaf(c.cmz, zm, r);
  r = fmaf(c.cpz, zp, r);
  return r;
}

// DPP wave shifts by one lane; the lane with no source reads zero (bound_ctrl)
__device__ __forceinline__ float lane_from_left(float v) {    // value of lane - 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v) {   // value of lane + 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

}  // namespace
