/*
 * oc.h -- C ABI of the compressed out-of-core stencil library (MI355X, gfx950).
 *
 * Method: Shen et al., "Compression-Based Optimizations for Out-of-Core GPU
 * Stencil Computation".  A field larger than device memory is split along z
 * into slabs that are streamed host -> device, advanced k time steps while
 * resident (temporal blocking: each slab carries k*r halo planes per side,
 * Sec. 3.1 and Sec. 3.2), and streamed back (Sec. 3.1).  With compression on,
 * the host keeps every slab compressed; the GPU decompresses after the
 * host-to-device copy and compresses before the device-to-host copy
 * (Sec. 1, Sec. 4.2), at a fixed user-specified rate (Sec. 5).  Three streams
 * share one full-size working buffer plus three compressed buffers (the single
 * working buffer method, Sec. 5); the conflict-free issue order follows
 * Algorithm 1 with the reading of its gaps documented in the design notes.
 *
 * Conventions shared by every call:
 *  - Return value: OC_OK (0) or a negative OC_ERR_* code; no exception or
 *    signal crosses this boundary (a host allocation failure inside the
 *    library returns OC_ERR_HOST, or 0 from the size queries).
 *    oc_status_str() names a code.
 *  - Arrays are FP32, C order [nz][ny][nx] (x fastest) unless stated.
 *  - Ownership: the caller allocates and outlives every large buffer (device
 *    arena, host levels, input/output arrays, streams).  The library owns only
 *    its handle, small metadata and HIP events.  The library never calls
 *    hipMalloc/hipHostMalloc.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are process memory (pinned memory makes copies asynchronous).
 *  - A handle is not thread-safe.  After OC_ERR_HIP (or OC_ERR_HOST from a
 *    call that queues work) the handle may only be destroyed; with two host levels the one that held the last complete
 *    sweep is intact (with in_place the level may be partly updated).
 *  - Ghost cells outside the grid are zero (zero Dirichlet boundary).
 */
#ifndef OC_H
#define OC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OC_OK = 0,
  OC_ERR_ARG = -1,       /* null pointer, non-positive size, out-of-range parameter     */
  OC_ERR_SHAPE = -2,     /* dims (or slab planes) not multiples of 4 with compression on */
  OC_ERR_BUDGET = -3,    /* the plan does not fit the device arena / host level sizes    */
  OC_ERR_HIP = -4,       /* a HIP runtime call failed (or an injected failure)            */
  OC_ERR_NONFINITE = -5, /* the codec met an Inf/NaN value                                */
  OC_ERR_STATE = -6,     /* call out of order (e.g. run before load)                      */
  OC_ERR_UNSUPPORTED = -7,
  OC_ERR_HOST = -8,      /* host memory or a host thread could not be had (C++ exception) */
  OC_ERR_TOO_LARGE = -9  /* input beyond the fixed scratch of an allocation-free entry point */
};

typedef struct oc_handle oc_handle;
typedef void *oc_stream; /* a hipStream_t (e.g. torch.cuda.Stream.cuda_stream) */

typedef struct { int64_t nx, ny, nz; } oc_grid;

typedef enum { OC_STAR7 = 1, OC_WAVE25 = 2 } oc_kind;

typedef struct {
  int32_t kind;          /* oc_kind                                                       */
  float c[7];            /* STAR7: c0, c_-x, c_+x, c_-y, c_+y, c_-z, c_+z                 */
  int32_t c0_is_field;   /* STAR7: 1 = c0 varies per cell, supplied as a field to oc_load  */
  float h, dt;           /* WAVE25: grid spacing (m) and time step (s)                    */
  int64_t src[3];        /* WAVE25: Ricker source cell (x, y, z); outside grid = none      */
  float f_peak, t0;      /* WAVE25: Ricker peak frequency (Hz) and delay (s)               */
} oc_stencil;

typedef struct {
  void *dev_arena;         /* device memory the library carves all buffers from             */
  size_t dev_budget;       /* its size in bytes; the plan must fit                          */
  oc_stream streams[3];    /* three caller-owned streams of default priority               */
  void *host_level[2];     /* two disjoint host buffers of >= oc_host_level_bytes() bytes
                              each (OC_ERR_ARG if they overlap; [1] unused with in_place);
                              pinned (hipHostMalloc / torch pin_memory) for overlap         */
  size_t host_level_bytes; /* size of each host level buffer                               */
  void *host_aux;          /* host buffer of >= oc_host_aux_bytes() bytes for the read-only
                              field (STAR7 c0 field, WAVE25 velocity); NULL when none       */
  size_t host_aux_bytes;   /* its size                                                      */
  int32_t k;               /* time steps per residency (temporal blocking), >= 1           */
  int32_t slab_planes;     /* S interior planes per slab; 0 = largest that fits the budget */
  int32_t rate_bits;       /* 0 = uncompressed; 1..32 = fixed-rate codec bits per value    */
  int32_t single_buffer;   /* compressed mode: 1 = one shared working buffer (Sec. 5),
                              0 = one working buffer per stream                            */
  int32_t timing;          /* 1 = time every kernel and copy of oc_run with HIP events
                              (results in oc_stats; costs two event records per op)         */
  int32_t ring_slots;      /* staging buffers in the copy ring, 2..8; 0 = 3 (Sec. 5)       */
  int32_t prefetch;        /* slabs copied in ahead of the kernels, 1..ring_slots-1;
                              0 = ring_slots - 1                                           */
  int32_t fuse_steps;      /* 7-point: time steps per stencil launch, 1..4 (one kernel
                              carries all of them through registers); 0 = 4                */
  int32_t copy_back;       /* device-to-host copies: n > 0 = a copy kernel of n workgroups
                              (1..1024) storing into the mapped pinned host pages; 0 = such a
                              kernel with 4 workgroups; -1 = the runtime's hipMemcpyAsync   */
  int32_t share_overlap;   /* region sharing (Sec. 3.1, Fig. 2): a slab takes the 2h planes
                              around its lower face from the previous slab's input on the
                              device instead of the host (coded runs of both stencils,
                              uncompressed 7-point runs with k <= fuse_steps, uncompressed
                              25-point runs through a per-slot stash of 2 x 2h planes that
                              the arena then holds; read-only c0 / velocity fields too);
                              0 or 1 = on where it applies, -1 = off (every slab loads both
                              halos).  Also applies to oc_adjoint's reverse sweeps.        */
  int32_t in_place;        /* 1 = one host level, host_level[0], updated in place by every
                              sweep (Algorithm 1, Ensure); host_level[1] is ignored and may
                              be NULL.  Needs region sharing in effect, or a single slab;
                              otherwise oc_create returns OC_ERR_ARG.  A run that fails
                              mid-sweep leaves that level partly updated.  0 = two levels
                              that alternate as source and destination                      */
  float error_budget;      /* > 0: the codec rate is chosen per error budget (7-point stencil;
                              else OC_ERR_UNSUPPORTED): oc_load runs the job's own process,
                              error_steps steps in residencies of k steps, each residency
                              decoding, stepping and re-encoding, on a z-sample of the loaded
                              field (whole xy planes, up to 64 planes from the middle of the
                              grid, zero beyond the sample) at candidate rates on the device,
                              beside the same steps uncompressed in FP32, and keeps the
                              smallest rate in 1..rate_bits whose relative L2 error is within
                              the budget (binary search: the error is taken to fall as the rate
                              rises).  rate_bits is then the largest rate allowed: host levels
                              and the arena are sized for it.  If no rate meets the budget,
                              rate_bits is used.  oc_stats reports the rate and the pilot's
                              error.  0 = the fixed rate rate_bits (Sec. 5)                  */
  int32_t error_steps;     /* the job length the budget is for (>= 1 with error_budget > 0)   */
  int32_t fused_codec;     /* 1 = each coded residency runs as one kernel (decode, k steps,
                              encode; no FP32 working buffer in device memory, the device
                              holds only the ring of coded slots): 7-point with constant c0,
                              k <= 4, rate_bits 1..16, else OC_ERR_UNSUPPORTED.  The codes
                              are those of the three-kernel path, bit for bit.  0 = decode,
                              stencil and encode kernels over a full-size working buffer   */
  int32_t load_rate_bits;  /* rate of the codes oc_load writes, which the first residency
                              after it decodes; every residency encodes at rate_bits, and
                              oc_store decodes the codes at the rate they were written.  A
                              field's roughest state is usually its first: after a few steps
                              the stencil has smoothed it and fewer bits keep the same error.
                              0 = rate_bits; else rate_bits..32 (with error_budget: the rate
                              picked, if that is higher), 7-point stencil without
                              fused_codec (else OC_ERR_UNSUPPORTED).  Host levels and ring
                              slots are sized for the larger of the two rates               */
} oc_config;

typedef struct {
  double wall_s;           /* wall time of the last oc_run                                 */
  double gcell_per_s;      /* nx*ny*nz*steps / wall_s / 1e9 of the last oc_run             */
  uint64_t bytes_h2d, bytes_d2h;  /* bytes copied by the last oc_run                       */
  uint64_t peak_dev_bytes; /* arena high-water mark of the plan (= device memory used)     */
  uint64_t slab_visits;    /* slabs processed by the last oc_run                           */
  int64_t slab_planes, halo_planes, n_slabs;  /* the plan                                  */
  uint64_t n_ops;          /* operations issued by the last oc_run                          */
  /* with timing on: summed durations (ms) and counts of the last oc_run's ops,
   * each measured between events recorded on the op's own stream; a fused
   * multi-step stencil launch counts once                                     */
  double ms_decode, ms_stencil, ms_encode, ms_h2d, ms_d2h;
  uint64_t n_decode, n_stencil, n_encode, n_h2d, n_d2h;
  uint64_t cells_stencil;  /* cell updates credited to the stencil launches               */
  uint64_t bytes_stencil;  /* algorithmic HBM bytes of those launches (input range read once,
                              output range written once, coefficient / velocity fields)    */
  uint64_t blocks_decode, blocks_encode;  /* 4x4x4 blocks coded                           */
  /* host wall time the last oc_run spent inside HIP calls: kernel launches
   * (including the copy-back kernel), host<->device copy calls, event record /
   * wait calls, and the final stream synchronisation (always measured)     */
  double host_ms_kernels, host_ms_copies, host_ms_events, host_ms_sync;
  int64_t rate_bits;       /* codec rate in use (0 = uncompressed); with an error budget, the
                              rate oc_load chose                                           */
  double pilot_rel_l2;     /* error budget: relative L2 error of the pilot at that rate       */
  int64_t pilot_planes;    /* error budget: planes of the z-sample the pilot ran on          */
  int64_t pilot_runs;      /* error budget: rates the last oc_load tried                     */
  double ms_fused;         /* timing on: summed durations of the fused codec launches        */
  uint64_t n_fused;        /* and their count                                                 */
} oc_stats;

/* Bytes one host level needs for this grid / stencil / rate (raw FP32 planes,
 * or z-major compressed block layers).  WAVE25 levels hold the two pressure
 * fields.  Returns 0 on bad arguments. */
size_t oc_host_level_bytes(const oc_grid *g, const oc_stencil *st, int32_t rate_bits);
/* Bytes of the read-only host field (STAR7 c0 field, WAVE25 velocity), coded
 * like a level; 0 when the stencil has none. */
size_t oc_host_aux_bytes(const oc_grid *g, const oc_stencil *st, int32_t rate_bits);

/* Bytes of device arena the plan for (g, st, cfg) needs; only the plan fields
 * of cfg are read (k, slab_planes, rate_bits, single_buffer, ring_slots,
 * prefetch; dev_budget caps the automatic slab depth, 0 = unlimited).
 * Returns 0 when no plan fits. */
size_t oc_plan_bytes(const oc_grid *g, const oc_stencil *st, const oc_config *cfg);

/* Plans the sweep (slab depth, halos, buffer carve-out, operation list) on the
 * CPU and creates HIP events.  Fails with OC_ERR_BUDGET when the buffers do not
 * fit dev_budget, OC_ERR_SHAPE when compression is on and nx, ny, nz or S are
 * not multiples of 4. */
int oc_create(const oc_grid *g, const oc_stencil *st, const oc_config *cfg, oc_handle **out);

/* Loads the initial state (host FP32 arrays, any host memory):
 *   STAR7:  u = field, aux = c0 field when c0_is_field (else NULL);
 *   WAVE25: u = p^0, aux = p^{-1}, vel = velocity (m/s).
 * With compression on, the fields are encoded on the GPU (the host keeps only
 * codes); the host level that holds no state (with two levels) then serves as
 * pinned staging for the caller's arrays and its contents are overwritten.
 * Synchronous. */
int oc_load(oc_handle *h, const float *u, const float *aux, const float *vel);

/* Advances the loaded state by `steps` time steps in sweeps of k steps (the
 * last sweep runs steps mod k when k does not divide steps).  Every sweep
 * streams all slabs through the GPU: H2D -> (decode) -> k stencil steps ->
 * (encode) -> D2H, pipelined over the three streams.  Synchronous: returns
 * after the three streams have drained. */
int oc_run(oc_handle *h, int64_t steps);

/* Copies the current state out (decoding on the GPU when compressed):
 *   STAR7: u; WAVE25: u = p^n, aux = p^{n-1} (either may be NULL).
 * With compression on and two host levels, the level not holding the current
 * state serves as pinned staging (overwritten).  Synchronous. */
int oc_store(oc_handle *h, float *u, float *aux);

int oc_stats_get(const oc_handle *h, oc_stats *s);
/* Turns the per-op timing of oc_run on (1) or off (0) after creation. */
int oc_set_timing(oc_handle *h, int32_t on);
int oc_destroy(oc_handle *h);

/* ---- fixed-rate codec on device buffers (Sec. 4.2, Sec. 5) -------------- */
/* Bytes of a compressed field: (nx/4)(ny/4)(nz/4) blocks of 8*rate_bits bytes.
 * Block (bx,by,bz) sits at byte ((bz*(ny/4) + by)*(nx/4) + bx) * 8*rate_bits,
 * so every group of 4 planes (a block layer) is one contiguous byte range. */
size_t oc_codec_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits);
/* Enqueues compression of d_in [nz][ny][nx] into d_out on `stream`; returns
 * after the enqueue.  Non-finite inputs set the stream's codec error word,
 * read by oc_codec_status.  The FP32 field must be 16-byte aligned and the
 * codes 4-byte aligned (as device allocations are); else OC_ERR_ARG. */
int oc_codec_compress(const float *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                      void *d_out, size_t out_bytes, oc_stream stream);
/* Enqueues decompression of the codes d_in into d_out [nz][ny][nx] FP32 on
 * `stream` (same alignment rules).  Every byte string of oc_codec_bytes()
 * bytes decodes, streams no encoder writes included: a block's stream ends at
 * its budget or where a run passes its last coefficient; large exponents give
 * infinities, never NaN. */
int oc_codec_decompress(const void *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                        float *d_out, oc_stream stream);
/* Synchronizes `stream` and returns OC_ERR_NONFINITE if any compression since
 * the last call met a non-finite value (and clears the flag), else OC_OK. */
int oc_codec_status(oc_stream stream);

/* Error of one codec round trip at rate_bits (Sec. 5: the error a fixed rate
 * costs), measured on the device without writing codes: every 4x4x4 block of
 * the FP32 field d_in [nz][ny][nx] (16-byte aligned, dims multiples of 4) is
 * encoded and decoded by one lane, and d_out (device, 3 doubles, 8-byte
 * aligned) receives sum (dec - in)^2, sum in^2 (FP64) and max |dec - in|.
 * Sums are taken in a fixed order (the same inputs give the same bits).
 * d_work: device scratch of >= oc_codec_error_work_bytes() bytes, 8-byte
 * aligned, owned by the caller.  Enqueued on `stream` (returns after the
 * enqueue); non-finite inputs set the flag oc_codec_status reports (the sums
 * are then meaningless). */
size_t oc_codec_error_work_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits);
int oc_codec_error(const float *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                   void *d_work, size_t work_bytes, double *d_out, oc_stream stream);

/* oc_codec_error without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and error behaviour as
 * oc_codec_error; the partial sums go to a static device array of just under
 * 2 MiB that each device holds until the process ends.  The call allocates
 * nothing (no hipMalloc, no allocating library routine).  Limit: at most
 * 87381 workgroups of the round-trip kernel, i.e. (nx/4)*(ny/4)*(nz/4) <=
 * 22,369,536 blocks for rate_bits <= 16 and <= 11,184,768 blocks above
 * (OC_ERR_TOO_LARGE beyond, checked on the host before anything is
 * enqueued).  The current device must own d_in, d_out and `stream`.  Every
 * call on a device shares that device's array (each call overwrites the sums
 * it reads, nothing needs clearing): calls that overlap on one device, e.g.
 * on two streams without ordering, race and give wrong sums. */
int oc_codec_error_noalloc(const float *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                           double *d_out, oc_stream stream);

/* ---- adjoint (differentiation of the 7-point path, raw handles) ---------- */
/* For u_T = A(c0)^T u_0 (A = the 7-point update with per-cell c0 when the
 * stencil has a c0 field), the gradients of a loss L(u_T) given dL/du_T:
 *   lambda_T = dL/du_T, lambda_n = A^T lambda_{n+1}  (A^T: -/+ coefficients
 *   swapped, the diagonal c0(x) kept), dL/du_0 = lambda_0,
 *   dL/dc0(x) = sum_n lambda_{n+1}(x) u_n(x).
 * oc_forward_ckpt advances the loaded state like oc_run(steps) and keeps the
 * states u_0, u_m, u_2m, ... (m = ckpt_every) in host_work, u_0 exact and the
 * others as codes at ckpt_rate_bits (0 = raw).  Those after u_0 are written by
 * the last sweep of each segment itself (encoded on the device from the slab
 * results) when the slab depth is a multiple of 4 or the checkpoints are raw,
 * and otherwise made from the host level between segments; the bytes are the
 * same either way.  oc_adjoint then runs reverse
 * sweeps, one per checkpoint segment, newest first: each slab reloads its
 * checkpoint, recomputes the segment's states in device memory and steps
 * lambda back while accumulating dL/dc0.  It may be called again with another
 * dL/du_T.  Both need a handle with rate_bits = 0.  host_work must hold
 * oc_adjoint_host_bytes() bytes (pinned for overlap) and outlive the calls. */
size_t oc_adjoint_host_bytes(const oc_handle *h, int64_t steps, int32_t ckpt_every,
                             int32_t ckpt_rate_bits);
int oc_forward_ckpt(oc_handle *h, int64_t steps, int32_t ckpt_every, int32_t ckpt_rate_bits,
                    void *host_work, size_t host_work_bytes);
/* gT, g_u0, g_c0: host FP32 [nz][ny][nx]; g_c0 may be NULL.  OC_ERR_STATE
 * unless oc_forward_ckpt has completed since the last oc_load (a load replaces
 * the state and the c0 field the checkpoints were taken from). */
int oc_adjoint(oc_handle *h, const float *gT, float *g_u0, float *g_c0);

/* ---- single-field device kernels (in-core building blocks) -------------- */
/* out = A^steps in on the device, ping-ponging through `tmp` (same size);
 * result lands in `out`.  c0f (nullable) is a device c0 field. */
int oc_star7_incore(const float *d_in, float *d_out, float *d_tmp, int64_t nx, int64_t ny,
                    int64_t nz, const float *c, const float *d_c0f, int64_t steps,
                    oc_stream stream);

/* Advances (p^{n0-1}, p^{n0}) = (d_prev, d_cur) by `steps` 25-point leapfrog
 * steps on the device (the Sec. 6 acoustic-wave update; WAVE25 stencil, Ricker
 * source of st).  On return d_cur holds p^{n0+steps}, d_prev p^{n0+steps-1};
 * d_tmp (same size) is needed when steps is odd, else may be NULL. */
int oc_wave25_incore(float *d_prev, float *d_cur, const float *d_vel, float *d_tmp, int64_t nx,
                     int64_t ny, int64_t nz, const oc_stencil *st, int64_t n0, int64_t steps,
                     oc_stream stream);

const char *oc_status_str(int status);

/* ---- stream check -------------------------------------------------------- */
/* Whether two streams run their kernels side by side.  The pipeline overlaps
 * the copy-back of one slab with the kernels of the next (Sec. 4.2, Fig. 4);
 * the copy-back is a kernel, so the kernel stream and the copy-back stream
 * must not be serialized.  The runtime maps streams onto a few hardware
 * queues in creation order, and two streams on one queue run in line; oc_run
 * cannot see that.  This runs a one-wave kernel of 2 ms (timed on the device's
 * constant-rate clock) on each stream at once, after a short first launch on
 * each, and writes into *overlap the share of the shorter run during which
 * both ran: about 1 when the streams run side by side, 0 when they are
 * serialized (for instance a == b).  Synchronizes both streams; the current
 * device must own both.  The two kernels record their clocks in one static
 * device array per device, so calls that overlap on one device race.
 * Errors: OC_ERR_ARG (null argument), OC_ERR_HIP. */
int oc_stream_overlap(oc_stream a, oc_stream b, double *overlap);

/* ---- test and debug hooks ----------------------------------------------- */
/* Makes the n-th HIP call issued by the executor from now on fail with
 * OC_ERR_HIP (n >= 1); n < 0 disables. */
int oc_debug_fail_after(oc_handle *h, int64_t n);
/* on != 0: the executor waits for all three streams after every operation it
 * issues (a run with no overlap at all, for comparing with the pipelined one);
 * 0 restores the pipeline. */
int oc_debug_serialize(oc_handle *h, int32_t on);
/* Builds the operation list of `sweeps` sweeps (k steps each) for the plan
 * of (g, st, cfg) (plan fields only, as oc_plan_bytes), without a GPU, and runs the happens-before checker
 * over it: returns the number of unordered conflicting accesses, plus
 * copy-ins that read host planes not last written by the previous sweep, plus
 * sweeps whose write-back does not cover the level (0 = race free, reads the
 * right state, complete), or a negative OC_ERR_* for a plan that cannot be made.
 * mutate: 0 none; 1 drop the i-th wait; 2 drop the epilogue (the last slab's
 * write-back); 3 swap op i with the next op of the same stream; 4 (in_place
 * plans) turn region sharing off, so slabs copy their halos from the level
 * being updated; 5 (two levels, sweeps >= 2) the second sweep copies in from
 * the level the first sweep read.  mutate = 0 with i = -1 returns the number
 * of waits instead. */
int64_t oc_debug_check_plan(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                            int64_t sweeps, int32_t mutate, int64_t i);
/* As oc_debug_check_plan, for the op list whose last sweep also writes the
 * new state to the checkpoint store (oc_forward_ckpt's segments): codes at
 * ckpt_rate_bits (1..32) or raw planes (0).  OC_ERR_UNSUPPORTED unless the
 * plan is an uncompressed 7-point plan (and, with codes, its slab interiors
 * are whole 4-plane block layers). */
int64_t oc_debug_check_plan_ckpt(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                                 int64_t sweeps, int32_t ckpt_rate_bits, int32_t mutate, int64_t i);
/* Writes a text listing of that operation list (one op per line) into buf
 * (truncated to len-1 bytes, NUL-terminated); returns the bytes the full
 * listing needs, or a negative OC_ERR_*. */
int64_t oc_debug_plan_dump(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                           int64_t sweeps, char *buf, size_t len);
/* The same checker over the reverse-sweep operation list of the adjoint for
 * `steps` steps with checkpoints every ckpt_every (mutate 0 or 1 as above).
 * With mutate = 0 and i = -1 it returns the number of waits instead. */
int64_t oc_debug_check_adjoint(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                               int64_t steps, int32_t ckpt_every, int32_t ckpt_rate_bits,
                               int32_t mutate, int64_t i);
/* Operations in that list; *n_waits receives the number of stream waits. */
int64_t oc_debug_plan_ops(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                          int64_t sweeps, int64_t *n_waits);

/* Enqueues on `stream` the copy-back kernel oc_run uses (copy_back > 0):
 * `workgroups` workgroups copy `bytes` from device memory at dev_src to byte
 * host_off of the pinned, mapped host allocation that starts at host_base
 * (OC_ERR_ARG if host_base is not the start of such memory; the caller keeps
 * host_off + bytes within it).  Returns after the enqueue.  Tuning aid: the
 * host-link probe measures this kernel's rate beside host-to-device DMA. */
int oc_debug_copy_to_host(void *host_base, size_t host_off, const void *dev_src, size_t bytes,
                          int32_t workgroups, oc_stream stream);

/* Tuning aid: one launch of the fused codec kernel (oc_config.fused_codec) on
 * device buffers, for a slab of out_nl interior block layers with one halo
 * layer on either side: d_in holds the slab's nl = out_nl + 2 layers of codes
 * at rate_bits (1..16) in the z-major block layout; layers [lay_lo, lay_hi)
 * are read, the others count as planes outside the grid (zeros); gz0 is the
 * global z of the slab's first plane (a multiple of 4, lay_lo / lay_hi and
 * the interior inside [0, nz)).  d_out receives the out_nl interior layers
 * after `steps` (1..4) 7-point steps with coefficients c[7], bit for bit the
 * codes of decode, steps and encode.  4-byte aligned device pointers; returns
 * after the enqueue on `stream`. */
int oc_debug_codec_star7(const void *d_in, void *d_out, int64_t nx, int64_t ny, int64_t nz, int64_t gz0,
                         int64_t out_nl, int64_t lay_lo, int64_t lay_hi, int32_t rate_bits, int32_t steps,
                         const float *c, oc_stream stream);

/* GPU timeline of the last oc_run (timing on): for each timed op, its class
 * (0 decode, 1 stencil, 2 encode, 3 host-to-device, 4 device-to-host), its
 * sweep * 100000 + slab, and its start / end in ms after the first timed op
 * started, from the op's own event pair.  With null arrays or cap <= 0,
 * returns the number of timed ops; else fills min(n, cap) entries and returns
 * that count.  Test and tuning aid. */
int64_t oc_debug_timeline(const oc_handle *h, int32_t *kind, int64_t *slab, double *start_ms,
                          double *end_ms, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
