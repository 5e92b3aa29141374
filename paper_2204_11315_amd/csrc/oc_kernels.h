// oc_kernels.h -- launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace oc {

// Optional per-launch timing: a launcher given a KernelTimer attaches its
// events to the first and last kernel it launches (hipExtLaunchKernel stamps
// them with those kernels' own start and end times, so no marker packets sit
// between the kernels) and sets `used`; a launcher that launches nothing
// leaves the events alone.
struct KernelTimer {
  hipEvent_t start = nullptr, stop = nullptr;
  bool used = false;
};
inline hipEvent_t kt_start(KernelTimer *kt) {
  if (!kt) return nullptr;
  kt->used = true;
  return kt->start;
}
inline hipEvent_t kt_stop(KernelTimer *kt) { return kt ? kt->stop : nullptr; }

// Fixed-rate codec over `nlayers` block layers (4 planes each) of an
// [4*nlayers][ny][nx] FP32 array; coded layers are contiguous.
hipError_t launch_encode(const float *d_in, int64_t nx, int64_t ny, int64_t nlayers, int rate,
                         void *d_out, hipStream_t s,
                         KernelTimer *kt = nullptr);
// d_in_lo (optional): the first lo_bytes of the coded input are read from
// there instead of from d_in (layers a slab shares with the previous one, left
// in that slab's staging slot); lo_bytes is a multiple of 4.
hipError_t launch_decode(const void *d_in, int64_t nx, int64_t ny, int64_t nlayers, int rate,
                         float *d_out, hipStream_t s,
                         KernelTimer *kt = nullptr, const void *d_in_lo = nullptr,
                         int64_t lo_bytes = 0);
// Device address of the codec's sticky error word.
hipError_t codec_error_word(int **dev_ptr);

// Round trip of the codec at `rate` over `nlayers` block layers of a device
// field, without writing codes: every block is encoded and decoded by one
// lane and compared with its inputs.  d_out3 (device) receives the sum of
// squared errors, the sum of squared inputs (FP64) and the largest absolute
// error; `parts` (device) holds codec_error_parts() triples of scratch.
// Non-finite inputs set the codec's error word.
int64_t codec_error_parts(int64_t nx, int64_t ny, int64_t nlayers, int rate);
hipError_t launch_codec_error(const float *d_in, int64_t nx, int64_t ny, int64_t nlayers, int rate,
                              double *parts, double *d_out3, hipStream_t s);
// The same three statistics of x against the reference ref over n values
// (n % 4 == 0, 16-byte aligned arrays); `parts` holds kDiffErrParts triples.
constexpr int64_t kDiffErrParts = 1024;
// Partial-sum triples the allocation-free round trip can hold (a static
// device array of 3 * kCodecErrStaticParts doubles, just under 2 MiB), and
// that array's address on the current device (looked up once per device).
constexpr int64_t kCodecErrStaticParts = 87381;
hipError_t codec_error_scratch(double **dev_ptr);
hipError_t launch_diff_error(const float *ref, const float *x, int64_t n, double *parts, double *d_out3,
                             hipStream_t s);

struct Star7Coef {
  float c0, cmx, cpx, cmy, cpy, cmz, cpz;
};

// One coded slab residency in one launch: decode the slot's block layers,
// `levels` (1..4) 7-point steps with constant coefficients, encode the
// interior.  in: local block layers [0, nl) of the slab (layers outside
// [lay_lo, lay_hi) are outside the grid and read as zero planes); out: the
// out_nl interior layers, starting at local layer out_l0 (the halo, >= 1
// layer and >= levels planes); nl = out_nl + 2 * out_l0.  The codes equal
// those of launch_decode, launch_star7_multi and launch_encode on the same
// slab.  Needs codec_star7_lds_bytes(rate) of LDS per workgroup.
constexpr int kCodecStar7MaxRate = 16;
size_t codec_star7_lds_bytes(int rate);
hipError_t launch_codec_star7(const void *in, void *out, int64_t nx, int64_t ny, int rate, int64_t lay_lo,
                              int64_t lay_hi, int64_t nl, int64_t out_l0, int64_t out_nl, int64_t gz0,
                              int64_t nz, int levels, const Star7Coef &c, hipStream_t s,
                              KernelTimer *kt = nullptr);

// One 7-point step on a slab buffer of `planes` planes whose local plane 0 is
// global plane gz0: writes local planes [z_lo, z_hi) of out from in.  Cells
// outside the global grid [0,nx) x [0,ny) x [0,nz) read as zero.  c0f
// (nullable) is the per-cell c0 slab with the same local indexing.
hipError_t launch_star7(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                        int64_t z_lo, int64_t z_hi, int64_t gz0, int64_t nz, const Star7Coef &c,
                        hipStream_t s,
                         KernelTimer *kt = nullptr);

// `levels` (1..4) fused 7-point steps: writes level `levels` on local planes
// [zo_lo, zo_hi) of out, reading in on [zo_lo - levels, zo_hi + levels).
// Bit-identical to `levels` single steps over shrinking ranges.
constexpr int kMaxFusedSteps = 4;
hipError_t launch_star7_multi(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                              int64_t zo_lo, int64_t zo_hi, int64_t gz0, int64_t nz, int levels,
                              const Star7Coef &c, hipStream_t s,
                         KernelTimer *kt = nullptr);

// g[i] += a[i] * b[i] for i < n.
hipError_t launch_axpy_prod(float *g, const float *a, const float *b, size_t n, hipStream_t s,
                         KernelTimer *kt = nullptr);

// One 25-point leapfrog step on a slab buffer (local plane 0 = global gz0):
// pnm1 <- 2 pn - pnm1 + (v dt/h)^2 L8(pn) on local planes [z_lo, z_hi), plus
// (v dt/h)^2 * src_amp at global cell src when it lies in that range.
hipError_t launch_wave25(const float *pn, float *pnm1, const float *vel, int64_t nx, int64_t ny,
                         int64_t z_lo, int64_t z_hi, int64_t gz0, int64_t nz, float dt_h,
                         const int64_t *src, float src_amp, hipStream_t s,
                         KernelTimer *kt = nullptr);

// Copies `bytes` from device memory into host memory that the device can
// address (pinned, mapped); a small grid so that it overlaps other kernels.
// Runs a 2 ms one-wave kernel on each of two streams at once and writes the
// share of the shorter one's run during which both ran (1: side by side, 0:
// one after the other).  Synchronizes both streams.
hipError_t probe_stream_overlap(hipStream_t a, hipStream_t b, double *overlap);
hipError_t launch_copy_to_host(void *dst, const void *src, size_t bytes, int workgroups, hipStream_t s,
                         KernelTimer *kt = nullptr);

}  // namespace oc
