// oc_plan.h -- slab planner, buffer carve-out and operation list (host only).
//
// The schedule is data: the planner emits a flat list of operations (copies,
// kernels, event records and waits) that the executor maps one-to-one onto HIP
// calls, and that the happens-before checker analyses on the CPU.  No HIP
// header is needed here.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace oc {

enum Kind { KIND_STAR7 = 1, KIND_WAVE25 = 2 };

// Storage ids of host memory an operation may touch.  The adjoint run maps
// the two levels to its two lambda levels and adds the checkpoint store and
// the coefficient-gradient store.
enum HostStore { HOST_LEVEL0 = 0, HOST_LEVEL1 = 1, HOST_AUX = 2, HOST_CKPT = 3, HOST_GRAD = 4 };
constexpr int kHostStores = 5;

enum OpType : uint8_t {
  OP_H2D,    // host store -> device arena           (host_id, host_off, dev_dst, bytes)
  OP_D2H,    // device arena -> host store           (dev_src, host_id, host_off, bytes)
  OP_DEC,    // codec decode: dev_src codes -> dev_dst planes (layers)
  OP_ENC,    // codec encode: dev_src planes -> dev_dst codes (layers)
  OP_STAR7,  // one 7-point step: dev_src -> dev_dst, local planes [z_lo, z_hi)
  OP_WAVE,   // one 25-point leapfrog step (dev_src = p^n, dev_dst = p^{n-1} -> p^{n+1})
  OP_AXPY,   // dev_dst[i] += dev_src[i] * dev_src2[i] over `bytes` bytes of FP32
  OP_REC,    // record event ev on stream
  OP_WAIT,   // stream waits for the latest record of ev
  OP_SYNC,   // host waits for every stream (end of a run)
  OP_ZERO,   // dev_dst[0, bytes) = 0 on the op's stream
  OP_FUSED   // coded slab in one kernel: dev_src = slot codes (local layer 0),
             // layers [z_lo, z_hi) hold codes; decode, `levels` 7-point steps,
             // encode the interior (`bytes` of codes) into dev_dst
};

struct Op {
  OpType type;
  int8_t stream;
  int8_t host_id;
  int32_t ev;
  int64_t dev_src, dev_src2, dev_dst;  // arena byte offsets (-1 = none)
  int64_t host_off, bytes;
  int64_t z_lo, z_hi;   // STAR7/WAVE: local planes updated; DEC/ENC: number of layers in z_hi
  int64_t gz0;          // global z of local plane 0 of the slab buffer
  int64_t planes;       // planes of the slab buffer (extent for the hazard model)
  int64_t step;         // WAVE: global time index n of p^n (source term)
  bool transpose;       // STAR7: apply A^T (the -/+ coefficients swapped)
  int32_t levels;       // STAR7: fused time steps in this launch (z_lo..z_hi = output planes)
  int32_t rate;         // DEC/ENC: bits per value when not the plan's (0 = the plan's)
  int32_t slab, sweep;  // bookkeeping (tests, stats)
};

struct Slab {
  int64_t z0, z1;   // interior global planes [z0, z1)
  int64_t l0, l1;   // loaded global planes [l0, l1) (clipped to the domain)
  int64_t gz0;      // global z of local plane 0 (= z0 - halo), may be negative
  int64_t planes;   // buffer planes used = (z1 - z0) + 2 * halo
};

struct PlanInput {
  int64_t nx = 0, ny = 0, nz = 0;
  int kind = KIND_STAR7;
  int k = 1;            // steps per residency
  int slab_planes = 0;  // 0 = automatic
  int rate = 0;         // 0 = raw
  bool single_buffer = true;
  bool c0_field = false;  // STAR7: a per-cell c0 slab rides along (raw)
  size_t budget = 0;      // 0 = unlimited
  int slots = 3;          // staging ring slots (2..8)
  int prefetch = -1;      // copy-ins issued ahead of the kernels (-1 = slots - 1)
  int fuse = 4;           // STAR7: time steps per stencil launch (1..kMaxFused)
  bool share = false;     // keep the overlap of consecutive slabs on the device
  bool in_place = false;  // one host level, updated in place (needs sharing or one slab)
  bool fused_codec = false;  // coded STAR7: one decode / k steps / encode kernel per slab
  int load_rate = 0;         // rate of the loaded codes (0 = rate), >= rate; STAR7, three kernels
};

constexpr int kMaxSlots = 8;
constexpr int kMaxFused = 4;   // time steps one 7-point launch may fuse

struct Plan {
  PlanInput in;
  int r = 1;               // stencil radius
  int64_t S = 0;           // interior planes per slab
  int64_t halo = 0;        // loaded halo planes per side (k*r rounded up to 4 when coded)
  int64_t P = 0;           // buffer planes = S + 2*halo
  bool coded = false;
  int n_rw = 1;            // read-write fields per level (STAR7 1, WAVE25 2)
  bool has_ro = false;     // read-only field streamed with every slab
  bool ro_coded = false;   // read-only field kept coded on the host
  size_t plane_bytes = 0;  // nx*ny*4
  size_t layer_bytes = 0;  // coded bytes of 4 planes
  int load_rate = 0;       // rate of the codes oc_load writes (= in.rate unless set)
  size_t max_layer_bytes = 0;   // coded bytes of 4 planes at the larger of the two rates
  bool share = false;      // region sharing in effect (STAR7; raw only with one stencil group)
  bool in_place = false;   // every sweep reads and writes host level 0
  int slots = 3;           // staging ring slots
  int prefetch = 2;        // copy-ins issued ahead
  int n_work_sets = 1;     // working-buffer sets (1 shared, or one per ring slot)
  // arena carve-out (byte offsets)
  size_t work_bytes = 0;   // one working buffer (P planes)
  size_t off_work[kMaxSlots][4] = {};   // [set][buffer]: STAR7 a, b, c0 ; WAVE25 v, pa, pb
  int n_work_bufs = 2;
  size_t stage_bytes = 0;  // one coded staging buffer
  size_t off_stage[kMaxSlots] = {};
  // fused codec: no working buffers; a slot holds the slab's input codes and,
  // at byte fused_out of the slot, the codes of its interior
  bool fused = false;
  size_t fused_out = 0;
  size_t off_ro_stage[kMaxSlots] = {};  // STAR7 raw c0 slab per ring slot (single working buffer)
  // WAVE25 raw with region sharing: per slot, the 2h planes of p^n and
  // p^{n-1} the next slab shares, set aside before the leapfrog overwrites them
  size_t stash_bytes = 0;
  size_t off_stash[kMaxSlots] = {};
  size_t arena_bytes = 0;
  std::vector<Slab> slabs;
  // host storage
  size_t host_field_bytes = 0;  // one field on the host (raw or coded)
  size_t host_level_bytes = 0;  // n_rw fields
  size_t host_aux_bytes = 0;
};

// Status codes mirror include/oc.h.
constexpr int ST_OK = 0, ST_ARG = -1, ST_SHAPE = -2, ST_BUDGET = -3, ST_UNSUPPORTED = -7;
// Highest rate the fused codec kernel takes (its LDS use grows with the rate).
constexpr int kFusedMaxRate = 16;

int stencil_radius(int kind);
size_t coded_layer_bytes(int64_t nx, int64_t ny, int rate);
// Builds the plan; returns a status.
int make_plan(const PlanInput &in, Plan *out);

// Streams of the schedule: copies in, kernels, copies out.
enum StreamRole { S_IN = 0, S_COMPUTE = 1, S_OUT = 2 };

// Event numbering for a plan with n slabs.  Slot q = g mod slots of the
// staging ring: "in" = its copy-in landed, "out" = its coded result is ready,
// "free" = its copy-back finished (the reverse sweeps of the adjoint; the
// forward op list uses the per-slab events for those two).  Per slab and sweep
// parity: copy-in / copy-back of that slab done.
struct EventIds {
  int n_slabs;
  int in(int q) const { return q; }
  int out(int q) const { return kMaxSlots + q; }
  int free(int q) const { return 2 * kMaxSlots + q; }
  int shr(int q) const { return 3 * kMaxSlots + q; }   // slot q's overlap copied onward
  int h2d(int parity, int j) const { return 4 * kMaxSlots + parity * n_slabs + j; }
  int d2h(int parity, int j) const { return 4 * kMaxSlots + 2 * n_slabs + parity * n_slabs + j; }
  int count() const { return 4 * kMaxSlots + 4 * n_slabs; }
};

// Operation list of `sweeps` consecutive sweeps starting from host level `src`
// (0 or 1).  steps_last = steps of the final sweep (<= k).  step0 = global
// time index at the start (WAVE25 source term).
// A copy of the state the last sweep of an op list writes, for a checkpoint
// store (HOST_CKPT): raw FP32 planes (rate 0) or codes at `rate`.  Raw
// 7-point plans whose slab interiors are whole block layers (or rate 0) only.
struct CkptOut {
  int rate = 0;
  size_t host_off = 0;   // byte offset of this checkpoint in the store
};
bool ckpt_out_supported(const Plan &p, int rate);
// rate0: the rate of the codes in host level `src` (the plan's load rate right
// after oc_load, its rate after any sweep; 0 = the plan's rate).  The first
// sweep copies and decodes them at that rate; every sweep encodes at the rate.
void build_ops(const Plan &p, int64_t sweeps, int steps_last, int src, int64_t step0,
               std::vector<Op> *ops, const CkptOut *ck = nullptr, int rate0 = 0);

// ---- adjoint (reverse sweeps over checkpoint segments) ------------------
// Forward states u_{s*m} (s = 0 .. nseg-1) are kept as checkpoints; segment s
// covers steps [s*m, min((s+1)*m, T)).  Per slab, the reverse of a segment
// loads the checkpoint, lambda_{n1}, c0 and the slab's coefficient-gradient
// interior, then for i = len-1 .. 0: recomputes u_{n0+i} from the checkpoint
// (i stencil steps on a range shrinking to the interior), adds
// lambda_{n0+i+1} * u_{n0+i} to the gradient, and steps lambda back with A^T.
struct AdjPlan {
  Plan g;                  // geometry (S, halo, P, slabs) and carve-out
  int m = 8;               // checkpoint interval
  int64_t steps = 0;       // T
  int nseg = 0;
  int ckpt_rate = 0;       // 0 = raw checkpoints
  // arena: per slot U0, La, Lb, Lc, C, G (P planes each) + coded stage; Wa and
  // Wb (kernel-only scratch of the recomputation) shared by the slots
  size_t off_buf[kMaxSlots][8] = {};
  size_t off_cstage[kMaxSlots] = {};
  // host checkpoint store: byte offset and coding of each checkpoint
  std::vector<size_t> ckpt_off;
  std::vector<int> ckpt_coded;
  size_t ckpt_bytes = 0;   // whole checkpoint store
  size_t field_bytes = 0;  // one raw field
};
enum AdjBuf { A_U0 = 0, A_WA, A_WB, A_LA, A_LB, A_C, A_G, A_LC };
// in: geometry input (kind STAR7, rate = ckpt rate for alignment, budget,
// slab_planes, share); m, T.  Returns a status.  With sharing, a slab after
// the first of its sweep takes the 2h planes around its lower face of the
// checkpoint state, lambda_{n1} and c0 from the previous slab's buffers (they
// stay intact: the recomputation writes Wa / Wb, lambda steps alternate
// between Lb and Lc) instead of the host.
int make_adj_plan(const PlanInput &in, int m, int64_t steps, AdjPlan *out);
// Reverse op list; lambda_T is read from host level `lsrc` (0/1); the final
// lambda_0 lands in level (lsrc + nseg) & 1.
void build_adjoint_ops(const AdjPlan &a, int lsrc, std::vector<Op> *ops);

// Human-readable listing of an operation list (one op per line).
std::string dump_ops(const std::vector<Op> &ops);

// Happens-before checker: number of pairs of conflicting accesses that are not
// ordered by stream order, event record/wait or host sync.  `why` (optional)
// receives a description of the first one.
int64_t check_ops(const Plan &p, const std::vector<Op> &ops, std::string *why,
                  bool check_writeback = true);

}  // namespace oc
