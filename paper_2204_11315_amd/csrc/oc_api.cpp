// oc_api.cpp -- the C ABI (include/oc.h) and the executor that maps the
// planner's operation list one-to-one onto HIP calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/oc.h"
#include "oc_kernels.h"
#include "oc_plan.h"

struct oc_handle {
  oc::Plan plan;
  oc_grid g;
  oc_stencil st;
  oc_config cfg;
  hipStream_t s[3];
  std::vector<hipEvent_t> ev;
  uint8_t *arena = nullptr;
  // host stores: level 0, level 1, aux, checkpoint store, gradient store
  uint8_t *host[oc::kHostStores] = {};
  // device view of each host store when it is pinned and mapped (copy-backs
  // then run as a small kernel), else nullptr (copy-backs use hipMemcpyAsync)
  uint8_t *host_dev[oc::kHostStores] = {};
  // adjoint: checkpoints of the last oc_forward_ckpt
  bool ckpt_valid = false;
  oc::AdjPlan adj;
  uint8_t *adj_work = nullptr;
  size_t adj_off[4] = {};   // checkpoint store, lambda A, lambda B, gradient store
  int cur = 0;            // host level holding the current state
  int level_rate = 0;     // rate of the codes in that level (the load rate after oc_load)
  bool loaded = false;
  bool broken = false;
  int64_t time_index = 0; // time steps applied since load
  oc_stats stats{};
  int64_t fail_after = -1;
  bool serialize = false;  // test hook: wait for every op before issuing the next
  int64_t hip_calls = 0;
  hipError_t last_hip = hipSuccess;
  // per-op timing (oc_config.timing)
  bool timing = false;
  std::vector<hipEvent_t> tev;
  // the last oc_run's timed ops: (kind, slab, index of its first event)
  struct TimedOp {
    int kind;
    int64_t slab;
    size_t ev;
  };
  std::vector<TimedOp> last_timed;
  // cached operation list
  std::vector<oc::Op> ops;
  int64_t ops_key[5] = {-1, -1, -1, -1, -1};
  // rate per error budget: the plan input at the largest rate (slab depth
  // pinned), replanned at the rate each oc_load picks
  bool auto_rate = false;
  oc::PlanInput in_max;
};

namespace {

// Large host copies and fills split over a few threads (one thread moves ~10
// GB/s; whole fields are GiBs, staged chunks tens of MiB).  Below 16 MiB the
// calling thread does it alone.
void par_bytes(void *dst, const void *src, size_t n) {   // src == nullptr: fill with zeros
  const size_t kMin = 8u << 20;
  unsigned t = std::min<unsigned>(8u, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 2 * kMin || t < 2) {
    if (src) std::memcpy(dst, src, n);
    else std::memset(dst, 0, n);
    return;
  }
  t = (unsigned)std::min<size_t>(t, n / kMin);
  const size_t per = (n / t + 4095) & ~(size_t)4095;
  std::vector<std::thread> pool;
  for (unsigned i = 0; i < t; i++) {
    const size_t lo = std::min(n, (size_t)i * per), hi = std::min(n, lo + per);
    if (lo >= hi) break;
    auto part = [=] {
      if (src) std::memcpy((uint8_t *)dst + lo, (const uint8_t *)src + lo, hi - lo);
      else std::memset((uint8_t *)dst + lo, 0, hi - lo);
    };
    try {
      pool.emplace_back(part);
    } catch (...) {   // no thread to be had: this part on the calling thread
      part();
    }
  }
  for (auto &th : pool) th.join();
}

thread_local hipError_t g_last_hip = hipSuccess;

// Every HIP call of the executor goes through here so that a test can inject a
// failure at the n-th call.
struct Exec {
  oc_handle *h;
  int st = OC_OK;
  bool ok(hipError_t e) {
    if (st != OC_OK) return false;
    if (h && h->fail_after > 0) {
      h->hip_calls++;
      if (h->hip_calls >= h->fail_after) {
        h->fail_after = -1;
        e = hipErrorUnknown;
      }
    }
    if (e != hipSuccess) {
      g_last_hip = e;
      if (h) h->last_hip = e;
      st = OC_ERR_HIP;
      return false;
    }
    return true;
  }
};

// Ricker wavelet (1 - 2 a) exp(-a), a = (pi f (t - t0))^2: the source term's
// time function, one scalar per step.
double ricker(double t, double f, double t0) {
  const double pi = 3.14159265358979323846;
  double a = pi * f * (t - t0);
  a *= a;
  return (1.0 - 2.0 * a) * std::exp(-a);
}

oc::Star7Coef coef_of(const oc_stencil &s) {
  return oc::Star7Coef{s.c[0], s.c[1], s.c[2], s.c[3], s.c[4], s.c[5], s.c[6]};
}

oc::PlanInput plan_input(const oc_grid *g, const oc_stencil *st, const oc_config *c) {
  oc::PlanInput in;
  in.nx = g->nx;
  in.ny = g->ny;
  in.nz = g->nz;
  in.kind = st->kind;
  in.k = c->k;
  in.slab_planes = c->slab_planes;
  in.rate = c->rate_bits;
  in.single_buffer = c->single_buffer != 0;
  in.c0_field = st->kind == OC_STAR7 && st->c0_is_field;
  in.budget = c->dev_budget;
  in.slots = c->ring_slots ? c->ring_slots : 3;
  in.prefetch = c->prefetch ? c->prefetch : -1;
  in.fuse = c->fuse_steps ? c->fuse_steps : oc::kMaxFused;
  in.share = c->share_overlap >= 0;
  in.in_place = c->in_place != 0;
  in.fused_codec = c->fused_codec != 0;
  in.load_rate = c->load_rate_bits;
  // with an error budget, rate_bits is the largest rate the pilot may pick:
  // the plan is sized for a load rate of at least that
  if (c->error_budget > 0.f && c->load_rate_bits > 0) in.load_rate = std::max(c->load_rate_bits, c->rate_bits);
  return in;
}

oc_config level_query_config(int32_t rate_bits) {
  oc_config c{};
  c.k = 1;
  c.slab_planes = 4;
  c.rate_bits = rate_bits;
  c.single_buffer = 1;
  return c;
}

void drain(oc_handle *h) {
  for (int i = 0; i < 3; i++) (void)hipStreamSynchronize(h->s[i]);
}

enum TimedKind { T_DEC, T_STENCIL, T_ENC, T_H2D, T_D2H, T_FUSED, T_NONE };
constexpr int kTimedKinds = T_NONE;

TimedKind timed_kind(const oc::Op &o) {
  switch (o.type) {
    case oc::OP_DEC: return o.z_hi < 0 ? T_NONE : T_DEC;
    case oc::OP_STAR7:
    case oc::OP_WAVE: return T_STENCIL;
    case oc::OP_ENC: return T_ENC;
    case oc::OP_H2D: return T_H2D;
    case oc::OP_D2H: return T_D2H;
    case oc::OP_FUSED: return T_FUSED;
    default: return T_NONE;
  }
}

int issue(oc_handle *h, const std::vector<oc::Op> &ops, const oc::Plan &p) {
  Exec x{h};
  const oc::Star7Coef c = coef_of(h->st);
  uint64_t h2d = 0, d2h = 0, cells = 0, bdec = 0, benc = 0, sbytes = 0;
  const uint64_t blocks_per_layer = (uint64_t)(p.in.nx / 4) * (uint64_t)(p.in.ny / 4);
  // timing: a pair of events around every timed op, recorded on its stream
  std::vector<std::pair<int, size_t>> timed;  // (kind, first event index)
  h->last_timed.clear();
  if (h->timing) {
    size_t need = 0;
    for (const oc::Op &o : ops) need += timed_kind(o) != T_NONE ? 2 : 0;
    while (h->tev.size() < need && x.st == OC_OK) {
      hipEvent_t e = nullptr;
      if (x.ok(hipEventCreate(&e))) h->tev.push_back(e);
    }
  }
  size_t tnext = 0;
  // host time spent inside the HIP calls of each op class
  enum { H_KERNEL, H_COPY, H_EVENT, H_SYNC, H_N };
  double host_s[H_N] = {0, 0, 0, 0};
  for (const oc::Op &o : ops) {
    hipStream_t s = o.stream >= 0 ? h->s[o.stream] : nullptr;
    const auto th0 = std::chrono::steady_clock::now();
    const TimedKind tk = h->timing ? timed_kind(o) : T_NONE;
    if (tk != T_NONE) {
      timed.push_back({(int)tk, tnext});
      h->last_timed.push_back({(int)tk, o.sweep * 100000 + o.slab, tnext});
    }
    // kernels carry their timing events themselves (stamped with the kernels'
    // own start / end); runtime copies are bracketed by marker events
    const bool kernel_d2h = o.type == oc::OP_D2H && h->host_dev[o.host_id] && h->cfg.copy_back >= 0;
    const bool marker_timed = tk != T_NONE && (o.type == oc::OP_H2D || (o.type == oc::OP_D2H && !kernel_d2h) ||
                                               (o.type == oc::OP_DEC && o.z_hi < 0));
    oc::KernelTimer ktimer;
    oc::KernelTimer *kt = nullptr;
    if (marker_timed) {
      x.ok(hipEventRecord(h->tev[tnext], s));
    } else if (tk != T_NONE) {
      ktimer.start = h->tev[tnext];
      ktimer.stop = h->tev[tnext + 1];
      kt = &ktimer;
    }
    switch (o.type) {
      case oc::OP_H2D:
        x.ok(hipMemcpyAsync(h->arena + o.dev_dst, h->host[o.host_id] + o.host_off, (size_t)o.bytes,
                            hipMemcpyHostToDevice, s));
        h2d += (uint64_t)o.bytes;
        break;
      case oc::OP_D2H:
        if (kernel_d2h)
          x.ok(oc::launch_copy_to_host(h->host_dev[o.host_id] + o.host_off, h->arena + o.dev_src,
                                       (size_t)o.bytes, h->cfg.copy_back, s, kt));
        else
          x.ok(hipMemcpyAsync(h->host[o.host_id] + o.host_off, h->arena + o.dev_src,
                              (size_t)o.bytes, hipMemcpyDeviceToHost, s));
        d2h += (uint64_t)o.bytes;
        break;
      case oc::OP_DEC:
        if (o.z_hi < 0) {
          x.ok(hipMemcpyAsync(h->arena + o.dev_dst, h->arena + o.dev_src, (size_t)o.bytes,
                              hipMemcpyDeviceToDevice, s));
        } else {
          // codes [0, bytes) from dev_src2 when set (shared layers where the
          // previous slab's copy-in left them)
          const bool two = o.dev_src2 >= 0 && o.bytes > 0;
          x.ok(oc::launch_decode(h->arena + o.dev_src, p.in.nx, p.in.ny, o.z_hi, o.rate > 0 ? o.rate : p.in.rate,
                                 (float *)(h->arena + o.dev_dst), s, kt,
                                 two ? h->arena + o.dev_src2 : nullptr, two ? o.bytes : 0));
          bdec += blocks_per_layer * (uint64_t)o.z_hi;
        }
        break;
      case oc::OP_ENC:
        x.ok(oc::launch_encode((const float *)(h->arena + o.dev_src), p.in.nx, p.in.ny, o.z_hi,
                               o.rate > 0 ? o.rate : p.in.rate, h->arena + o.dev_dst, s, kt));
        benc += blocks_per_layer * (uint64_t)o.z_hi;
        break;
      case oc::OP_STAR7: {
        // A^T: the neighbour coefficients swap direction, the diagonal stays
        const oc::Star7Coef ct{c.c0, c.cpx, c.cmx, c.cpy, c.cmy, c.cpz, c.cmz};
        const float *c0p = o.dev_src2 >= 0 ? (const float *)(h->arena + o.dev_src2) : nullptr;
        if (o.levels > 1)
          x.ok(oc::launch_star7_multi((const float *)(h->arena + o.dev_src), (float *)(h->arena + o.dev_dst),
                                      c0p, p.in.nx, p.in.ny, o.z_lo, o.z_hi, o.gz0, p.in.nz, o.levels,
                                      o.transpose ? ct : c, s, kt));
        else
          x.ok(oc::launch_star7((const float *)(h->arena + o.dev_src), (float *)(h->arena + o.dev_dst),
                                c0p, p.in.nx, p.in.ny, o.z_lo, o.z_hi, o.gz0, p.in.nz,
                                o.transpose ? ct : c, s, kt));
        {
          // credited cell updates: levels x output planes; algorithmic bytes:
          // the input range read once, the output range written once (+ c0)
          const uint64_t pc = (uint64_t)p.in.nx * (uint64_t)p.in.ny;
          const uint64_t out_planes = (uint64_t)(o.z_hi - o.z_lo);
          const uint64_t in_planes = out_planes + 2u * (uint64_t)(o.levels * p.r);
          cells += (uint64_t)o.levels * out_planes * pc;
          sbytes += 4u * pc * (in_planes + out_planes + (c0p ? in_planes : 0u));
        }
        break;
      }
      case oc::OP_ZERO:
        x.ok(hipMemsetAsync(h->arena + o.dev_dst, 0, (size_t)o.bytes, s));
        break;
      case oc::OP_FUSED: {
        const int64_t nl = o.planes / 4, out_l0 = p.halo / 4;
        x.ok(oc::launch_codec_star7(h->arena + o.dev_src, h->arena + o.dev_dst, p.in.nx, p.in.ny, p.in.rate,
                                    o.z_lo, o.z_hi, nl, out_l0, nl - 2 * out_l0, o.gz0, p.in.nz, o.levels, c,
                                    s, kt));
        const uint64_t out_layers = (uint64_t)(nl - 2 * out_l0);
        bdec += blocks_per_layer * (uint64_t)(o.z_hi - o.z_lo);
        benc += blocks_per_layer * out_layers;
        cells += (uint64_t)o.levels * out_layers * 4u * (uint64_t)p.in.nx * (uint64_t)p.in.ny;
        break;
      }
      case oc::OP_AXPY:
        x.ok(oc::launch_axpy_prod((float *)(h->arena + o.dev_dst), (const float *)(h->arena + o.dev_src),
                                  (const float *)(h->arena + o.dev_src2), (size_t)o.bytes / 4u, s, kt));
        break;
      case oc::OP_WAVE: {
        const float amp = (float)ricker((double)o.step * h->st.dt, h->st.f_peak, h->st.t0);
        x.ok(oc::launch_wave25((const float *)(h->arena + o.dev_src), (float *)(h->arena + o.dev_dst),
                               (const float *)(h->arena + o.dev_src2), p.in.nx, p.in.ny, o.z_lo,
                               o.z_hi, o.gz0, p.in.nz, h->st.dt / h->st.h, h->st.src, amp, s, kt));
        cells += (uint64_t)(o.z_hi - o.z_lo) * (uint64_t)p.in.nx * (uint64_t)p.in.ny;
        sbytes += 16u * (uint64_t)(o.z_hi - o.z_lo) * (uint64_t)p.in.nx * (uint64_t)p.in.ny;
        break;
      }
      case oc::OP_REC:
      case oc::OP_WAIT:
        if (o.ev < 0 || (size_t)o.ev >= h->ev.size()) {
          x.st = OC_ERR_STATE;   // an event the handle does not own: never issue it
          break;
        }
        if (o.type == oc::OP_REC)
          x.ok(hipEventRecord(h->ev[o.ev], s));
        else
          x.ok(hipStreamWaitEvent(s, h->ev[o.ev], 0));
        break;
      case oc::OP_SYNC:
        for (int i = 0; i < 3; i++) x.ok(hipStreamSynchronize(h->s[i]));
        break;
    }
    if (tk != T_NONE) {
      if (marker_timed) {
        x.ok(hipEventRecord(h->tev[tnext + 1], s));
      } else if (!ktimer.used) {   // nothing was launched: an empty interval
        x.ok(hipEventRecord(h->tev[tnext], s));
        x.ok(hipEventRecord(h->tev[tnext + 1], s));
      }
      tnext += 2;
    }
    {
      int hc = H_KERNEL;
      switch (o.type) {
        case oc::OP_H2D: hc = H_COPY; break;
        case oc::OP_D2H: hc = h->host_dev[o.host_id] && h->cfg.copy_back >= 0 ? H_KERNEL : H_COPY; break;
        case oc::OP_REC:
        case oc::OP_WAIT: hc = H_EVENT; break;
        case oc::OP_SYNC: hc = H_SYNC; break;
        default: break;
      }
      host_s[hc] += std::chrono::duration<double>(std::chrono::steady_clock::now() - th0).count();
    }
    if (h->serialize && x.st == OC_OK && o.type != oc::OP_SYNC)
      for (int i = 0; i < 3; i++) x.ok(hipStreamSynchronize(h->s[i]));
    if (x.st != OC_OK) break;
  }
  h->stats.host_ms_kernels = host_s[H_KERNEL] * 1e3;
  h->stats.host_ms_copies = host_s[H_COPY] * 1e3;
  h->stats.host_ms_events = host_s[H_EVENT] * 1e3;
  h->stats.host_ms_sync = host_s[H_SYNC] * 1e3;
  h->stats.bytes_h2d = h2d;
  h->stats.bytes_d2h = d2h;
  h->stats.cells_stencil = cells;
  h->stats.bytes_stencil = sbytes;
  h->stats.blocks_decode = bdec;
  h->stats.blocks_encode = benc;
  double ms[kTimedKinds] = {};
  uint64_t n[kTimedKinds] = {};
  if (x.st == OC_OK && h->timing) {
    for (const auto &t : timed) {
      float e = 0.f;
      if (!x.ok(hipEventElapsedTime(&e, h->tev[t.second], h->tev[t.second + 1]))) break;
      ms[t.first] += e;
      n[t.first]++;
    }
  }
  h->stats.ms_decode = ms[T_DEC];
  h->stats.ms_stencil = ms[T_STENCIL];
  h->stats.ms_encode = ms[T_ENC];
  h->stats.ms_h2d = ms[T_H2D];
  h->stats.ms_d2h = ms[T_D2H];
  h->stats.n_decode = n[T_DEC];
  h->stats.n_stencil = n[T_STENCIL];
  h->stats.n_encode = n[T_ENC];
  h->stats.n_h2d = n[T_H2D];
  h->stats.n_d2h = n[T_D2H];
  h->stats.ms_fused = ms[T_FUSED];
  h->stats.n_fused = n[T_FUSED];
  if (x.st != OC_OK) {
    drain(h);
    h->broken = true;
  }
  return x.st;
}

int codec_check_and_clear() {
  int *w = nullptr;
  if (oc::codec_error_word(&w) != hipSuccess || !w) return OC_ERR_HIP;
  int v = 0;
  if (hipMemcpy(&v, w, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return OC_ERR_HIP;
  if (v) {
    int z = 0;
    if (hipMemcpy(w, &z, sizeof z, hipMemcpyHostToDevice) != hipSuccess) return OC_ERR_HIP;
    return OC_ERR_NONFINITE;
  }
  return OC_OK;
}

// Device address of pinned, mapped host memory, or nullptr.
uint8_t *mapped_host(void *p) {
  if (!p) return nullptr;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  return (uint8_t *)a.devicePointer;
}

bool grid_ok(const oc_grid *g) {
  return g && g->nx > 0 && g->ny > 0 && g->nz > 0 && g->nx <= (1 << 30) && g->ny <= (1 << 30) &&
         g->nz <= (1 << 30);
}

// A free pinned host region that can stage a caller's pageable field: the
// host level that holds no state (none when one level is updated in place),
// if it fits two chunks of `chunk` planes; else nullptr.
uint8_t *bounce_region(const oc_handle *h, int free_level, int64_t chunk) {
  const oc::Plan &p = h->plan;
  if (p.in_place || !h->host[free_level]) return nullptr;
  const size_t need = 2u * (size_t)chunk * p.plane_bytes;
  return h->cfg.host_level_bytes >= need ? h->host[free_level] : nullptr;
}

// Encodes a whole host FP32 field into host codes at `rate`, in chunks of
// `chunk` planes, double-buffered through two device buffer pairs (raw
// `work[i]`, codes `stage[i]`): the copy-in of a chunk (stream 0) overlaps the
// encode (stream 1) and copy-back (stream 2) of the one before.  With a pinned
// `bounce` region (two chunks), each chunk is first copied there by host
// threads while the previous one crosses the link (pageable sources copy in
// far slower than pinned ones).  Returns when the codes are on the host.
int encode_field(oc_handle *h, const float *src, uint8_t *dst, int rate, int64_t chunk,
                 uint8_t *const work[2], uint8_t *const stage[2], uint8_t *bounce = nullptr) {
  const oc::Plan &p = h->plan;
  Exec x{h};
  const size_t pb = p.plane_bytes;
  const size_t layer = oc::coded_layer_bytes(p.in.nx, p.in.ny, rate);
  const size_t half = (size_t)chunk * pb;
  hipEvent_t ev[6] = {};   // per buffer pair: copied in, encoded, copied back
  for (auto &e : ev)
    if (!x.ok(hipEventCreateWithFlags(&e, hipEventDisableTiming))) break;
  int64_t c = 0;
  for (int64_t z = 0; z < p.in.nz && x.st == OC_OK; z += chunk, c++) {
    const int b = (int)(c & 1);
    const int64_t n = std::min<int64_t>(chunk, p.in.nz - z);
    if (c >= 2) x.ok(hipStreamWaitEvent(h->s[0], ev[3 * b + 2], 0));   // pair b copied back
    const uint8_t *from = (const uint8_t *)src + (size_t)z * pb;
    if (bounce && x.st == OC_OK) {
      // half b was last read by the copy-in of chunk c - 2
      if (c >= 2 && !x.ok(hipEventSynchronize(ev[3 * b]))) break;
      par_bytes(bounce + b * half, from, (size_t)n * pb);
      from = bounce + b * half;
    }
    x.ok(hipMemcpyAsync(work[b], from, (size_t)n * pb, hipMemcpyHostToDevice, h->s[0]));
    x.ok(hipEventRecord(ev[3 * b], h->s[0]));
    x.ok(hipStreamWaitEvent(h->s[1], ev[3 * b], 0));
    x.ok(oc::launch_encode((const float *)work[b], p.in.nx, p.in.ny, n / 4, rate, stage[b], h->s[1]));
    x.ok(hipEventRecord(ev[3 * b + 1], h->s[1]));
    x.ok(hipStreamWaitEvent(h->s[2], ev[3 * b + 1], 0));
    x.ok(hipMemcpyAsync(dst + (size_t)(z / 4) * layer, stage[b], (size_t)(n / 4) * layer,
                        hipMemcpyDeviceToHost, h->s[2]));
    x.ok(hipEventRecord(ev[3 * b + 2], h->s[2]));
  }
  // drain every stream (also after an error: the buffers must be idle)
  for (int i = 0; i < 3; i++) (void)hipStreamSynchronize(h->s[i]);
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  if (x.st) return x.st;
  return codec_check_and_clear();
}

// Device buffers oc_load / oc_store stage a coded field through: two FP32
// chunks (`work`) and their codes (`stage`); returns the chunk in planes.
// Three-kernel plans use the working buffers and staging slots 0 and 1 (P
// planes per chunk); fused plans, which have no FP32 buffers, carve the
// chunks from the arena: the largest multiple of 4 planes whose two FP32
// chunks and two code chunks fit it (the planner sizes the arena for >= 4).
int64_t io_buffers(const oc_handle *h, uint8_t *work[2], uint8_t *stage[2]) {
  const oc::Plan &p = h->plan;
  if (!p.fused) {
    work[0] = h->arena + p.off_work[0][0];
    work[1] = h->arena + (p.n_work_sets == 1 ? p.off_work[0][1] : p.off_work[1][0]);
    stage[0] = h->arena + p.off_stage[0];
    stage[1] = h->arena + p.off_stage[1];
    return std::max<int64_t>(4, p.P / 4 * 4);
  }
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  auto need = [&](int64_t c) {
    return 2u * up((size_t)c * p.plane_bytes) + 2u * up((size_t)(c / 4) * p.layer_bytes);
  };
  int64_t c = 4;
  while (c + 4 <= (p.in.nz + 3) / 4 * 4 && need(c + 4) <= p.arena_bytes) c += 4;
  const size_t fb = up((size_t)c * p.plane_bytes), cb = up((size_t)(c / 4) * p.layer_bytes);
  work[0] = h->arena;
  work[1] = h->arena + fb;
  stage[0] = h->arena + 2 * fb;
  stage[1] = h->arena + 2 * fb + cb;
  return c;
}

// Loads a host FP32 field into host store `dst`: a copy, or codes at the
// plan's rate made on the GPU through the plan's first working and staging
// buffers.
int load_field(oc_handle *h, const float *src, uint8_t *dst, bool coded) {
  const oc::Plan &p = h->plan;
  if (!coded) {
    par_bytes(dst, src, p.plane_bytes * (size_t)p.in.nz);
    return OC_OK;
  }
  uint8_t *work[2], *stage[2];
  const int64_t chunk = io_buffers(h, work, stage);
  // level 0 receives the codes (at the load rate); level 1 holds nothing yet
  return encode_field(h, src, dst, p.load_rate, chunk, work, stage, bounce_region(h, 1, chunk));
}

// Host store `src` back to a host FP32 field: a copy, or the codes decoded on
// the GPU, double-buffered over the three streams like encode_field (codes in,
// decode, field out) through the plan's first two working and staging buffers.
// With a free pinned level, each chunk lands there and host threads move it to
// `dst` while the next one is decoded and copied out.
int store_field(oc_handle *h, const uint8_t *src, float *dst, bool coded) {
  const oc::Plan &p = h->plan;
  const size_t pb = p.plane_bytes;
  const int rate = coded ? (h->level_rate > 0 ? h->level_rate : p.in.rate) : 0;
  const size_t lb = coded ? oc::coded_layer_bytes(p.in.nx, p.in.ny, rate) : 0;
  if (!coded) {
    par_bytes(dst, src, pb * (size_t)p.in.nz);
    return OC_OK;
  }
  Exec x{h};
  uint8_t *work[2], *stage[2];
  const int64_t chunk = io_buffers(h, work, stage);
  uint8_t *const bounce = bounce_region(h, 1 - h->cur, chunk);
  const size_t half = (size_t)chunk * pb;
  hipEvent_t ev[6] = {};   // per buffer pair: codes in, decoded, copied out
  for (auto &e : ev)
    if (!x.ok(hipEventCreateWithFlags(&e, hipEventDisableTiming))) break;
  // moves chunk c (planes [z, z + n)) from its bounce half to dst once copied out
  auto drain = [&](int64_t c, int64_t z, int64_t n) {
    const int b = (int)(c & 1);
    if (x.ok(hipEventSynchronize(ev[3 * b + 2])))
      par_bytes((uint8_t *)dst + (size_t)z * pb, bounce + b * half, (size_t)n * pb);
  };
  int64_t c = 0, zp = 0, np = 0;   // the chunk before c
  for (int64_t z = 0; z < p.in.nz && x.st == OC_OK; z += chunk, c++) {
    const int b = (int)(c & 1);
    const int64_t n = std::min<int64_t>(chunk, p.in.nz - z);
    if (c >= 2) x.ok(hipStreamWaitEvent(h->s[0], ev[3 * b + 2], 0));   // pair b copied out
    x.ok(hipMemcpyAsync(stage[b], src + (size_t)(z / 4) * lb, (size_t)(n / 4) * lb, hipMemcpyHostToDevice,
                        h->s[0]));
    x.ok(hipEventRecord(ev[3 * b], h->s[0]));
    x.ok(hipStreamWaitEvent(h->s[1], ev[3 * b], 0));
    x.ok(oc::launch_decode(stage[b], p.in.nx, p.in.ny, n / 4, rate, (float *)work[b], h->s[1]));
    x.ok(hipEventRecord(ev[3 * b + 1], h->s[1]));
    x.ok(hipStreamWaitEvent(h->s[2], ev[3 * b + 1], 0));
    uint8_t *to = bounce ? bounce + b * half : (uint8_t *)dst + (size_t)z * pb;
    x.ok(hipMemcpyAsync(to, work[b], (size_t)n * pb, hipMemcpyDeviceToHost, h->s[2]));
    x.ok(hipEventRecord(ev[3 * b + 2], h->s[2]));
    // the previous chunk's half is written to again only by chunk c + 1,
    // which is queued after this returns
    if (bounce && c >= 1 && x.st == OC_OK) drain(c - 1, zp, np);
    zp = z;
    np = n;
  }
  if (bounce && c >= 1 && x.st == OC_OK) drain(c - 1, zp, np);
  // drain every stream (also after an error: the buffers must be idle)
  for (int i = 0; i < 3; i++) (void)hipStreamSynchronize(h->s[i]);
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  return x.st;
}

// ---- codec rate per error budget ------------------------------------------
// The job's own process (error_steps steps in residencies of k: decode, k
// stencil steps, encode; the field encoded first and decoded last) runs on a
// z-sample of the loaded field, whole xy planes, beside the same steps
// uncompressed in FP32; the relative L2 difference at a rate is the pilot's
// prediction of the job's error at that rate.  The sample is its own grid:
// zero beyond its first and last plane.
struct PilotLayout {
  int64_t planes = 0;
  size_t u0 = 0, ref = 0, x = 0, y = 0, c0 = 0, codes = 0, parts = 0, out = 0, need = 0;
};

PilotLayout pilot_layout(const oc::PlanInput &in, int64_t planes) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t fb = up((size_t)planes * (size_t)in.nx * (size_t)in.ny * 4u);
  PilotLayout L;
  L.planes = planes;
  size_t o = 0;
  L.u0 = o, o += fb;
  L.ref = o, o += fb;
  L.x = o, o += fb;
  L.y = o, o += fb;
  if (in.c0_field) L.c0 = o, o += fb;
  L.codes = o, o += up((size_t)(planes / 4) * oc::coded_layer_bytes(in.nx, in.ny, std::max(in.rate, in.load_rate)));
  L.parts = o, o += up((size_t)oc::kDiffErrParts * 3u * sizeof(double));
  L.out = o, o += up(3u * sizeof(double));
  L.need = o;
  return L;
}

constexpr int64_t kPilotMaxPlanes = 64;

// Planes of the pilot's z-sample that fit `bytes` of device memory (up to
// kPilotMaxPlanes, a multiple of 4; 0 if not even 4 fit).
int64_t pilot_planes_within(const oc::PlanInput &in, size_t bytes) {
  int64_t planes = std::min<int64_t>(kPilotMaxPlanes, in.nz / 4 * 4);
  while (planes >= 4 && pilot_layout(in, planes).need > bytes) planes -= 4;
  return planes >= 4 ? planes : 0;
}

// Device bytes a handle needs: the plan's arena, and with an error budget at
// least the pilot's largest sample within `budget` (the pilot runs in the
// arena during oc_load, before the job uses it).
size_t arena_bytes_for(const oc::Plan &p, const oc_config *cfg) {
  if (!(cfg->error_budget > 0.f)) return p.arena_bytes;
  const int64_t planes = pilot_planes_within(p.in, cfg->dev_budget);
  if (planes == 0) return p.arena_bytes;
  return std::max(p.arena_bytes, pilot_layout(p.in, planes).need);
}

// Picks the rate for the field u (c0f: the c0 field, or nullptr), replans the
// handle at that rate and records the choice in its stats.
int pick_rate(oc_handle *h, const float *u, const float *c0f) {
  const oc::PlanInput &in = h->in_max;
  const int rmax = in.rate;
  const int64_t nx = in.nx, ny = in.ny, nz = in.nz;
  const int64_t planes = pilot_planes_within(in, h->cfg.dev_budget);
  if (planes < 4) return OC_ERR_BUDGET;
  const PilotLayout L = pilot_layout(in, planes);
  const size_t pb = (size_t)nx * (size_t)ny * 4u;
  const int64_t z0 = (nz - planes) / 2 / 4 * 4;
  uint8_t *A = h->arena;
  float *U0 = (float *)(A + L.u0), *RF = (float *)(A + L.ref), *X = (float *)(A + L.x),
        *Y = (float *)(A + L.y);
  const float *C0 = c0f ? (const float *)(A + L.c0) : nullptr;
  uint8_t *CD = A + L.codes;
  double *parts = (double *)(A + L.parts), *dout = (double *)(A + L.out);
  hipStream_t s = h->s[1];
  Exec x{h};
  x.ok(hipMemcpyAsync(U0, (const uint8_t *)u + (size_t)z0 * pb, (size_t)planes * pb, hipMemcpyHostToDevice, s));
  if (c0f)
    x.ok(hipMemcpyAsync(A + L.c0, (const uint8_t *)c0f + (size_t)z0 * pb, (size_t)planes * pb,
                        hipMemcpyHostToDevice, s));
  const oc::Star7Coef c = coef_of(h->st);
  // n steps from src, alternating between a and b (a != src); the result's buffer
  auto steps_on = [&](const float *src, int64_t n, float *a, float *b) {
    const float *cur = src;
    float *dst = a;
    while (n > 0 && x.st == OC_OK) {
      const int lv = (int)std::min<int64_t>(n, oc::kMaxFusedSteps);
      x.ok(oc::launch_star7_multi(cur, dst, C0, nx, ny, 0, planes, 0, planes, lv, c, s));
      cur = dst;
      dst = dst == a ? b : a;
      n -= lv;
    }
    return cur;
  };
  const int64_t steps = h->cfg.error_steps, k = in.k;
  const float *r = steps_on(U0, steps, X, Y);
  x.ok(hipMemcpyAsync(RF, r, (size_t)planes * pb, hipMemcpyDeviceToDevice, s));
  const int64_t layers = planes / 4;
  std::vector<double> err((size_t)rmax + 1, -1.0);
  int runs = 0;
  // the loaded field is encoded at the load rate (at least R), the residencies at R
  const int load_user = h->cfg.load_rate_bits;
  auto run = [&](int R) -> double {
    if (err[(size_t)R] >= 0.0) return err[(size_t)R];
    int rin = std::max(load_user, R);
    x.ok(oc::launch_encode(U0, nx, ny, layers, rin, CD, s));
    for (int64_t done = 0; done < steps && x.st == OC_OK;) {
      const int64_t n = std::min<int64_t>(k, steps - done);
      x.ok(oc::launch_decode(CD, nx, ny, layers, rin, X, s));
      rin = R;
      const float *res = steps_on(X, n, Y, X);
      x.ok(oc::launch_encode(res, nx, ny, layers, R, CD, s));
      done += n;
    }
    x.ok(oc::launch_decode(CD, nx, ny, layers, rin, X, s));
    x.ok(oc::launch_diff_error(RF, X, planes * nx * ny, parts, dout, s));
    double sums[3] = {0.0, 0.0, 0.0};
    x.ok(hipMemcpyAsync(sums, dout, sizeof sums, hipMemcpyDeviceToHost, s));
    x.ok(hipStreamSynchronize(s));
    runs++;
    const double e = sums[1] > 0.0 ? std::sqrt(sums[0] / sums[1]) : (sums[0] > 0.0 ? HUGE_VAL : 0.0);
    err[(size_t)R] = e;
    return e;
  };
  // smallest rate within the budget, by bisection over 1..rmax
  const double budget = (double)h->cfg.error_budget;
  int best = -1;
  for (int lo = 1, hi = rmax; lo <= hi && x.st == OC_OK;) {
    const int mid = (lo + hi) / 2;
    if (run(mid) <= budget) {
      best = mid;
      hi = mid - 1;
    } else {
      lo = mid + 1;
    }
  }
  if (x.st != OC_OK) {
    drain(h);
    return x.st;
  }
  if (best < 0) best = rmax;
  const double best_err = run(best);
  if (x.st != OC_OK) return x.st;
  const int cr = codec_check_and_clear();
  if (cr) return cr;
  oc::PlanInput pin = in;
  pin.rate = best;
  pin.load_rate = load_user > 0 ? std::max(load_user, best) : 0;
  oc::Plan np;
  const int pr = oc::make_plan(pin, &np);
  if (pr != oc::ST_OK) return pr;
  if (np.arena_bytes > h->cfg.dev_budget || np.slabs.size() != h->plan.slabs.size()) return OC_ERR_BUDGET;
  h->plan = np;
  std::memset(h->ops_key, 0xff, sizeof h->ops_key);   // cached ops belong to the old rate
  h->stats.peak_dev_bytes = std::max(np.arena_bytes, L.need);   // the pilot ran in the arena too
  h->stats.rate_bits = best;
  h->stats.pilot_rel_l2 = best_err;
  h->stats.pilot_planes = planes;
  h->stats.pilot_runs = runs;
  return OC_OK;
}

}  // namespace

extern "C" {

const char *oc_status_str(int st) {
  switch (st) {
    case OC_OK: return "ok";
    case OC_ERR_ARG: return "invalid argument";
    case OC_ERR_SHAPE: return "shape not block aligned (multiples of 4 needed with compression)";
    case OC_ERR_BUDGET: return "plan does not fit the device budget or host buffers";
    case OC_ERR_HIP: return hipGetErrorString(g_last_hip);
    case OC_ERR_NONFINITE: return "non-finite value met by the codec";
    case OC_ERR_STATE: return "call out of order";
    case OC_ERR_UNSUPPORTED: return "unsupported combination";
    case OC_ERR_HOST: return "host allocation or thread creation failed";
    case OC_ERR_TOO_LARGE: return "input larger than the allocation-free entry point's fixed scratch";
    default: return "unknown status";
  }
}

size_t oc_codec_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits) {
  try {
    if (nx <= 0 || ny <= 0 || nz <= 0 || rate_bits < 1 || rate_bits > 32) return 0;
    if (nx % 4 || ny % 4 || nz % 4) return 0;
    return (size_t)(nx / 4) * (size_t)(ny / 4) * (size_t)(nz / 4) * 8u * (size_t)rate_bits;
  } catch (...) {
    return 0;
  }
}

int oc_codec_compress(const float *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                      void *d_out, size_t out_bytes, oc_stream stream) {
  try {
    if (!d_in || !d_out || nx <= 0 || ny <= 0 || nz <= 0 || rate_bits < 1 || rate_bits > 32)
      return OC_ERR_ARG;
    // the kernels move the field as float4s and the codes as dwords
    if (((uintptr_t)d_in & 15) || ((uintptr_t)d_out & 3)) return OC_ERR_ARG;
    if (nx % 4 || ny % 4 || nz % 4) return OC_ERR_SHAPE;
    if (out_bytes < oc_codec_bytes(nx, ny, nz, rate_bits)) return OC_ERR_ARG;
    hipError_t e = oc::launch_encode(d_in, nx, ny, nz / 4, rate_bits, d_out, (hipStream_t)stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_codec_decompress(const void *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                        float *d_out, oc_stream stream) {
  try {
    if (!d_in || !d_out || nx <= 0 || ny <= 0 || nz <= 0 || rate_bits < 1 || rate_bits > 32)
      return OC_ERR_ARG;
    if (((uintptr_t)d_in & 3) || ((uintptr_t)d_out & 15)) return OC_ERR_ARG;
    if (nx % 4 || ny % 4 || nz % 4) return OC_ERR_SHAPE;
    hipError_t e = oc::launch_decode(d_in, nx, ny, nz / 4, rate_bits, d_out, (hipStream_t)stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_codec_status(oc_stream stream) {
  try {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return codec_check_and_clear();
  } catch (...) {
    return OC_ERR_HOST;
  }
}

size_t oc_codec_error_work_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits) {
  try {
    if (nx <= 0 || ny <= 0 || nz <= 0 || rate_bits < 1 || rate_bits > 32) return 0;
    if (nx % 4 || ny % 4 || nz % 4) return 0;
    return (size_t)oc::codec_error_parts(nx, ny, nz / 4, rate_bits) * 3u * sizeof(double);
  } catch (...) {
    return 0;
  }
}

int oc_codec_error(const float *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                   void *d_work, size_t work_bytes, double *d_out, oc_stream stream) {
  try {
    if (!d_in || !d_work || !d_out || nx <= 0 || ny <= 0 || nz <= 0 || rate_bits < 1 || rate_bits > 32)
      return OC_ERR_ARG;
    if (((uintptr_t)d_in & 15) || ((uintptr_t)d_work & 7) || ((uintptr_t)d_out & 7)) return OC_ERR_ARG;
    if (nx % 4 || ny % 4 || nz % 4) return OC_ERR_SHAPE;
    if (work_bytes < oc_codec_error_work_bytes(nx, ny, nz, rate_bits)) return OC_ERR_ARG;
    hipError_t e = oc::launch_codec_error(d_in, nx, ny, nz / 4, rate_bits, (double *)d_work, d_out,
                                          (hipStream_t)stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_codec_error_noalloc(const float *d_in, int64_t nx, int64_t ny, int64_t nz, int32_t rate_bits,
                           double *d_out, oc_stream stream) {
  try {
    if (!d_in || !d_out || nx <= 0 || ny <= 0 || nz <= 0 || rate_bits < 1 || rate_bits > 32)
      return OC_ERR_ARG;
    if (((uintptr_t)d_in & 15) || ((uintptr_t)d_out & 7)) return OC_ERR_ARG;
    if (nx % 4 || ny % 4 || nz % 4) return OC_ERR_SHAPE;
    if (oc::codec_error_parts(nx, ny, nz / 4, rate_bits) > oc::kCodecErrStaticParts)
      return OC_ERR_TOO_LARGE;
    double *parts = nullptr;
    hipError_t e = oc::codec_error_scratch(&parts);
    if (e == hipSuccess)
      e = oc::launch_codec_error(d_in, nx, ny, nz / 4, rate_bits, parts, d_out, (hipStream_t)stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_star7_incore(const float *d_in, float *d_out, float *d_tmp, int64_t nx, int64_t ny,
                    int64_t nz, const float *c, const float *d_c0f, int64_t steps,
                    oc_stream stream) {
  try {
    if (!d_in || !d_out || !c || nx <= 0 || ny <= 0 || nz <= 0 || steps < 0) return OC_ERR_ARG;
    if (((uintptr_t)d_in | (uintptr_t)d_out | (uintptr_t)d_tmp | (uintptr_t)d_c0f) & 3) return OC_ERR_ARG;
    if (steps > oc::kMaxFusedSteps && !d_tmp) return OC_ERR_ARG;
    if (nx > (1 << 30) || ny > (1 << 30) || nz > (1 << 30)) return OC_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    oc::Star7Coef cf{c[0], c[1], c[2], c[3], c[4], c[5], c[6]};
    hipError_t e = hipSuccess;
    if (steps == 0) {
      e = hipMemcpyAsync(d_out, d_in, (size_t)(nx * ny * nz) * 4u, hipMemcpyDeviceToDevice, s);
    } else {
      // groups of up to kMaxFusedSteps fused steps, ping-ponging so that the
      // last group writes d_out
      const int64_t groups = (steps + oc::kMaxFusedSteps - 1) / oc::kMaxFusedSteps;
      float *X = (groups % 2 == 1) ? d_out : d_tmp;
      float *Y = (groups % 2 == 1) ? d_tmp : d_out;
      const float *src = d_in;
      int64_t done = 0;
      for (int64_t gi = 1; gi <= groups && e == hipSuccess; gi++) {
        const int lv = (int)std::min<int64_t>(oc::kMaxFusedSteps, steps - done);
        float *dst = (gi % 2 == 1) ? X : Y;
        e = lv > 1 ? oc::launch_star7_multi(src, dst, d_c0f, nx, ny, 0, nz, 0, nz, lv, cf, s)
                   : oc::launch_star7(src, dst, d_c0f, nx, ny, 0, nz, 0, nz, cf, s);
        src = dst;
        done += lv;
      }
    }
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_wave25_incore(float *d_prev, float *d_cur, const float *d_vel, float *d_tmp, int64_t nx,
                     int64_t ny, int64_t nz, const oc_stencil *st, int64_t n0, int64_t steps,
                     oc_stream stream) {
  try {
    if (!d_prev || !d_cur || !d_vel || !st || nx <= 0 || ny <= 0 || nz <= 0 || steps < 0 || n0 < 0)
      return OC_ERR_ARG;
    if (st->kind != OC_WAVE25 || !(st->h > 0.f && st->dt > 0.f)) return OC_ERR_ARG;
    if (((uintptr_t)d_prev | (uintptr_t)d_cur | (uintptr_t)d_vel | (uintptr_t)d_tmp) & 3) return OC_ERR_ARG;
    if (nx > (1 << 30) || ny > (1 << 30) || nz > (1 << 30)) return OC_ERR_ARG;
    if ((steps & 1) && !d_tmp) return OC_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    float *a = d_prev, *b = d_cur;   // a holds p^{n-1}, b holds p^n
    for (int64_t i = 0; i < steps && e == hipSuccess; i++) {
      const float amp = (float)ricker((double)(n0 + i) * st->dt, st->f_peak, st->t0);
      e = oc::launch_wave25(b, a, d_vel, nx, ny, 0, nz, 0, nz, st->dt / st->h, st->src, amp, s);
      std::swap(a, b);
    }
    if (e == hipSuccess && (steps & 1)) {
      // the newest level is in d_prev: swap the two buffers' contents
      const size_t bytes = (size_t)(nx * ny * nz) * 4u;
      e = hipMemcpyAsync(d_tmp, d_prev, bytes, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(d_prev, d_cur, bytes, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(d_cur, d_tmp, bytes, hipMemcpyDeviceToDevice, s);
    }
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

size_t oc_host_level_bytes(const oc_grid *g, const oc_stencil *st, int32_t rate_bits) {
  try {
    if (!grid_ok(g) || !st) return 0;
    oc::Plan p;
    oc_config c = level_query_config(rate_bits);
    if (oc::make_plan(plan_input(g, st, &c), &p) != oc::ST_OK) return 0;
    return p.host_level_bytes;
  } catch (...) {
    return 0;
  }
}

size_t oc_host_aux_bytes(const oc_grid *g, const oc_stencil *st, int32_t rate_bits) {
  try {
    if (!grid_ok(g) || !st) return 0;
    oc::Plan p;
    oc_config c = level_query_config(rate_bits);
    if (oc::make_plan(plan_input(g, st, &c), &p) != oc::ST_OK) return 0;
    return p.host_aux_bytes;
  } catch (...) {
    return 0;
  }
}

size_t oc_plan_bytes(const oc_grid *g, const oc_stencil *st, const oc_config *cfg) {
  try {
    if (!grid_ok(g) || !st || !cfg) return 0;
    oc::Plan p;
    if (oc::make_plan(plan_input(g, st, cfg), &p) != oc::ST_OK) return 0;
    return arena_bytes_for(p, cfg);
  } catch (...) {
    return 0;
  }
}

int oc_create(const oc_grid *g, const oc_stencil *st, const oc_config *cfg, oc_handle **out) {
  try {
    if (!grid_ok(g) || !st || !cfg || !out) return OC_ERR_ARG;
    *out = nullptr;
    if (st->kind != OC_STAR7 && st->kind != OC_WAVE25) return OC_ERR_ARG;
    if (st->kind == OC_WAVE25 && !(st->h > 0.f && st->dt > 0.f)) return OC_ERR_ARG;
    if (cfg->copy_back < -1 || cfg->copy_back > 1024) return OC_ERR_ARG;
    const bool auto_rate = cfg->error_budget > 0.f;
    if (auto_rate) {
      if (st->kind != OC_STAR7) return OC_ERR_UNSUPPORTED;
      if (!std::isfinite(cfg->error_budget) || cfg->rate_bits < 1 || cfg->rate_bits > 32 ||
          cfg->error_steps < 1)
        return OC_ERR_ARG;
    } else if (cfg->error_budget < 0.f || std::isnan(cfg->error_budget)) {
      return OC_ERR_ARG;
    }
    oc::Plan p;
    int r = oc::make_plan(plan_input(g, st, cfg), &p);
    if (r != oc::ST_OK) return r;
    if (!cfg->dev_arena || p.arena_bytes > cfg->dev_budget) return OC_ERR_BUDGET;
    if (!cfg->host_level[0] || (!p.in_place && !cfg->host_level[1]) ||
        cfg->host_level_bytes < p.host_level_bytes)
      return OC_ERR_BUDGET;
    if (!p.in_place) {   // two levels: each sweep reads one and writes the other
      const uintptr_t a = (uintptr_t)cfg->host_level[0], b = (uintptr_t)cfg->host_level[1];
      const uintptr_t n = (uintptr_t)p.host_level_bytes;
      if (a < b + n && b < a + n) return OC_ERR_ARG;
    }
    if (p.host_aux_bytes && (!cfg->host_aux || cfg->host_aux_bytes < p.host_aux_bytes))
      return OC_ERR_BUDGET;
    for (int i = 0; i < 3; i++)
      if (!cfg->streams[i]) return OC_ERR_ARG;
    std::unique_ptr<oc_handle> owner(new oc_handle());
    oc_handle *h = owner.get();
    h->plan = p;
    h->g = *g;
    h->st = *st;
    h->cfg = *cfg;
    for (int i = 0; i < 3; i++) h->s[i] = (hipStream_t)cfg->streams[i];
    h->timing = cfg->timing != 0;
    h->arena = (uint8_t *)cfg->dev_arena;
    h->host[0] = (uint8_t *)cfg->host_level[0];
    h->host[1] = p.in_place ? nullptr : (uint8_t *)cfg->host_level[1];
    h->host[2] = (uint8_t *)cfg->host_aux;
    for (int i = 0; i < 3; i++) h->host_dev[i] = mapped_host(h->host[i]);
    h->ckpt_valid = false;
    oc::EventIds ids{(int)p.slabs.size()};
    h->ev.assign((size_t)ids.count(), nullptr);
    for (auto &e : h->ev) {
      hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
      if (err != hipSuccess) {
        g_last_hip = err;
        for (auto &f : h->ev)
          if (f) (void)hipEventDestroy(f);
        return OC_ERR_HIP;
      }
    }
    h->stats.peak_dev_bytes = p.arena_bytes;
    h->stats.rate_bits = p.in.rate;
    h->auto_rate = auto_rate;
    h->in_max = p.in;
    h->in_max.slab_planes = (int)p.S;   // the slabs stay those planned for the largest rate
    h->stats.slab_planes = p.S;
    h->stats.halo_planes = p.halo;
    h->stats.n_slabs = (int64_t)p.slabs.size();
    *out = owner.release();
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_load(oc_handle *h, const float *u, const float *aux, const float *vel) {
  try {
    if (!h || !u) return OC_ERR_ARG;
    if (h->broken) return OC_ERR_STATE;
    const oc::Plan &p = h->plan;
    const bool wave = p.in.kind == oc::KIND_WAVE25;
    if (p.in.c0_field && !aux) return OC_ERR_ARG;
    if (wave && (!aux || !vel)) return OC_ERR_ARG;
    // the checkpoints of an earlier oc_forward_ckpt belong to the old state
    // and c0 field (the reverse sweeps read c0 from the aux store reloaded
    // here): oc_adjoint needs a new forward
    h->ckpt_valid = false;
    h->cur = 0;
    if (h->auto_rate) {
      const int pr = pick_rate(h, u, p.in.c0_field ? aux : nullptr);
      if (pr) {
        h->broken = pr == OC_ERR_HIP;
        return pr;
      }
    }
    int r = load_field(h, u, h->host[0], p.coded);
    if (!r && wave) r = load_field(h, aux, h->host[0] + p.host_field_bytes, p.coded);
    if (!r && wave) r = load_field(h, vel, h->host[2], p.ro_coded);
    if (r) {
      h->broken = r == OC_ERR_HIP;
      return r;
    }
    if (p.in.c0_field) par_bytes(h->host[2], aux, (size_t)p.host_aux_bytes);
    h->level_rate = p.coded ? p.load_rate : 0;
    h->loaded = true;
    h->time_index = 0;
    return OC_OK;
  } catch (...) {
    if (h) h->broken = true;
    return OC_ERR_HOST;
  }
}

namespace {

// `steps` time steps through the pipeline; with `ck`, the last sweep also
// writes the new state to the checkpoint store (that op list is not cached).
int run_steps(oc_handle *h, int64_t steps, const oc::CkptOut *ck) {
  const oc::Plan &p = h->plan;
  const int64_t k = p.in.k;
  const int64_t sweeps = (steps + k - 1) / k;
  const int steps_last = (int)(steps - (sweeps - 1) * k);
  const int64_t t_key = p.in.kind == oc::KIND_WAVE25 ? h->time_index : 0;
  const int rate0 = p.coded ? h->level_rate : 0;
  int64_t key[5] = {sweeps, steps_last, h->cur, t_key, rate0};
  if (ck) {
    oc::build_ops(p, sweeps, steps_last, h->cur, h->time_index, &h->ops, ck, rate0);
    std::memset(h->ops_key, 0xff, sizeof h->ops_key);   // not a valid key
  } else if (std::memcmp(key, h->ops_key, sizeof key) != 0) {
    oc::build_ops(p, sweeps, steps_last, h->cur, h->time_index, &h->ops, nullptr, rate0);
    std::memcpy(h->ops_key, key, sizeof key);
  }
  auto t0 = std::chrono::steady_clock::now();
  int r = issue(h, h->ops, h->plan);
  auto t1 = std::chrono::steady_clock::now();
  if (r) return r;
  int cr = p.coded ? codec_check_and_clear() : OC_OK;
  if (!p.in_place) h->cur = (int)((h->cur + sweeps) & 1);
  if (p.coded) h->level_rate = p.in.rate;   // every sweep encodes at the rate
  h->time_index += steps;
  double wall = std::chrono::duration<double>(t1 - t0).count();
  h->stats.wall_s = wall;
  h->stats.gcell_per_s =
      (double)p.in.nx * (double)p.in.ny * (double)p.in.nz * (double)steps / wall / 1e9;
  h->stats.slab_visits = (uint64_t)(sweeps * (int64_t)p.slabs.size());
  h->stats.n_ops = h->ops.size();
  return cr;
}

}  // namespace

int oc_run(oc_handle *h, int64_t steps) {
  try {
    if (!h || steps < 0) return OC_ERR_ARG;
    if (h->broken || !h->loaded) return OC_ERR_STATE;
    if (steps == 0) return OC_OK;
    return run_steps(h, steps, nullptr);
  } catch (...) {
    if (h) h->broken = true;
    return OC_ERR_HOST;
  }
}

int oc_store(oc_handle *h, float *u, float *aux) {
  try {
    if (!h || (!u && !aux)) return OC_ERR_ARG;
    if (h->broken || !h->loaded) return OC_ERR_STATE;
    const oc::Plan &p = h->plan;
    int r = OC_OK;
    if (u) r = store_field(h, h->host[h->cur], u, p.coded);
    if (!r && aux && p.in.kind == oc::KIND_WAVE25)
      r = store_field(h, h->host[h->cur] + p.host_field_bytes, aux, p.coded);
    return r;
  } catch (...) {
    if (h) h->broken = true;
    return OC_ERR_HOST;
  }
}

// ---- adjoint ------------------------------------------------------------
namespace {

size_t align4k(size_t x) { return (x + 4095) & ~(size_t)4095; }

// Grows the handle's event pool to n events.
int ensure_events(oc_handle *h, size_t n) {
  while (h->ev.size() < n) {
    hipEvent_t e = nullptr;
    hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
    if (err != hipSuccess) {
      g_last_hip = err;
      return OC_ERR_HIP;
    }
    h->ev.push_back(e);
  }
  return OC_OK;
}

int adj_plan_for(const oc_handle *h, int64_t steps, int32_t every, int32_t rate, oc::AdjPlan *a) {
  if (h->plan.in.kind != oc::KIND_STAR7) return OC_ERR_UNSUPPORTED;
  if (h->plan.coded) return OC_ERR_UNSUPPORTED;     // the forward of the adjoint runs raw
  if (steps < 1 || every < 1 || rate < 0 || rate > 32) return OC_ERR_ARG;
  oc::PlanInput in = h->plan.in;
  in.in_place = false;    // the reverse sweeps keep their own two lambda levels
  in.rate = rate;
  in.slab_planes = 0;
  in.budget = h->cfg.dev_budget;
  int r = oc::make_adj_plan(in, every, steps, a);
  return r;
}

size_t adj_work_bytes(const oc::AdjPlan &a, size_t *off) {
  size_t o = 0;
  off[0] = o;
  o = align4k(o + a.ckpt_bytes);
  for (int i = 1; i < 4; i++) {
    off[i] = o;
    o = align4k(o + a.field_bytes);
  }
  return o;
}

}  // namespace

size_t oc_adjoint_host_bytes(const oc_handle *h, int64_t steps, int32_t ckpt_every,
                             int32_t ckpt_rate_bits) {
  try {
    if (!h) return 0;
    oc::AdjPlan a;
    if (adj_plan_for(h, steps, ckpt_every, ckpt_rate_bits, &a) != OC_OK) return 0;
    size_t off[4];
    return adj_work_bytes(a, off);
  } catch (...) {
    return 0;
  }
}

int oc_forward_ckpt(oc_handle *h, int64_t steps, int32_t ckpt_every, int32_t ckpt_rate_bits,
                    void *host_work, size_t host_work_bytes) {
  try {
    if (!h || !host_work) return OC_ERR_ARG;
    if (h->broken || !h->loaded) return OC_ERR_STATE;
    oc::AdjPlan a;
    int r = adj_plan_for(h, steps, ckpt_every, ckpt_rate_bits, &a);
    if (r != OC_OK) return r;
    size_t off[4];
    if (adj_work_bytes(a, off) > host_work_bytes) return OC_ERR_BUDGET;
    h->ckpt_valid = false;
    uint8_t *work = (uint8_t *)host_work;
    // Checkpoint sg + 1 is written by the last sweep of segment sg itself
    // (codes made from the slab results on the device) where the plan allows;
    // otherwise, and for u_0, it is made from the host level between segments.
    const bool in_pipe = oc::ckpt_out_supported(h->plan, a.ckpt_rate);
    uint8_t *const saved = h->host[oc::HOST_CKPT], *const saved_dev = h->host_dev[oc::HOST_CKPT];
    h->host[oc::HOST_CKPT] = work + off[0];
    h->host_dev[oc::HOST_CKPT] = mapped_host(work + off[0]);
    for (int sg = 0; sg < a.nseg && r == OC_OK; sg++) {
      if (sg == 0 || !in_pipe) {
        uint8_t *dst = work + off[0] + a.ckpt_off[(size_t)sg];
        const float *cur = (const float *)h->host[h->cur];
        if (a.ckpt_coded[(size_t)sg]) {
          // codes made on the GPU through the adjoint plan's two slots' buffers
          uint8_t *const wbuf[2] = {h->arena + a.off_buf[0][oc::A_U0], h->arena + a.off_buf[1][oc::A_U0]};
          uint8_t *const sbuf[2] = {h->arena + a.off_cstage[0], h->arena + a.off_cstage[1]};
          r = encode_field(h, cur, dst, a.ckpt_rate, std::max<int64_t>(4, a.g.P / 4 * 4), wbuf, sbuf);
        } else {
          par_bytes(dst, cur, a.field_bytes);
        }
        if (r) {
          h->broken = r == OC_ERR_HIP;
          break;
        }
      }
      const int64_t len = std::min<int64_t>(ckpt_every, steps - (int64_t)sg * ckpt_every);
      oc::CkptOut ck;
      const bool next = in_pipe && sg + 1 < a.nseg;
      if (next) {
        ck.rate = a.ckpt_coded[(size_t)sg + 1] ? a.ckpt_rate : 0;
        ck.host_off = a.ckpt_off[(size_t)sg + 1];
      }
      r = run_steps(h, len, next ? &ck : nullptr);
      if (!r && next && ck.rate > 0) r = codec_check_and_clear();
    }
    h->host[oc::HOST_CKPT] = saved;
    h->host_dev[oc::HOST_CKPT] = saved_dev;
    if (r) return r;
    h->adj = a;
    h->adj_work = work;
    std::memcpy(h->adj_off, off, sizeof off);
    h->ckpt_valid = true;
    return OC_OK;
  } catch (...) {
    if (h) h->broken = true;
    return OC_ERR_HOST;
  }
}

int oc_adjoint(oc_handle *h, const float *gT, float *g_u0, float *g_c0) {
  try {
    if (!h || !gT || !g_u0) return OC_ERR_ARG;
    if (h->broken) return OC_ERR_STATE;
    if (!h->ckpt_valid) return OC_ERR_STATE;
    const oc::AdjPlan &a = h->adj;
    uint8_t *w = h->adj_work;
    uint8_t *lam0 = w + h->adj_off[1], *lam1 = w + h->adj_off[2], *grad = w + h->adj_off[3];
    // (the gradient store is not cleared: the first reverse sweep starts each
    // slab's accumulator at zero on the device and writes the whole store)
    par_bytes(lam0, gT, a.field_bytes);
    // map the host stores of the reverse sweeps, run them, restore the handle's
    uint8_t *saved[oc::kHostStores], *saved_dev[oc::kHostStores];
    std::memcpy(saved, h->host, sizeof saved);
    std::memcpy(saved_dev, h->host_dev, sizeof saved_dev);
    h->host[0] = lam0;
    h->host[1] = lam1;
    h->host[oc::HOST_CKPT] = w + h->adj_off[0];
    h->host[oc::HOST_GRAD] = grad;
    for (int i : {0, 1, (int)oc::HOST_CKPT, (int)oc::HOST_GRAD}) h->host_dev[i] = mapped_host(h->host[i]);
    const int er = ensure_events(h, (size_t)oc::EventIds{(int)a.g.slabs.size()}.count());
    if (er) {
      std::memcpy(h->host, saved, sizeof saved);
      std::memcpy(h->host_dev, saved_dev, sizeof saved_dev);
      return er;
    }
    std::vector<oc::Op> ops;
    oc::build_adjoint_ops(a, 0, &ops);
    auto t0 = std::chrono::steady_clock::now();
    int r = issue(h, ops, a.g);
    auto t1 = std::chrono::steady_clock::now();
    std::memcpy(h->host, saved, sizeof saved);
    std::memcpy(h->host_dev, saved_dev, sizeof saved_dev);
    if (r) return r;
    if (a.ckpt_rate > 0) {
      int cr = codec_check_and_clear();
      if (cr) return cr;
    }
    h->stats.wall_s = std::chrono::duration<double>(t1 - t0).count();
    h->stats.n_ops = ops.size();
    par_bytes(g_u0, (a.nseg & 1) ? lam1 : lam0, a.field_bytes);
    if (g_c0) par_bytes(g_c0, grad, a.field_bytes);
    return OC_OK;
  } catch (...) {
    if (h) h->broken = true;
    return OC_ERR_HOST;
  }
}

int64_t oc_debug_check_adjoint(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                               int64_t steps, int32_t ckpt_every, int32_t ckpt_rate_bits,
                               int32_t mutate, int64_t i) {
  try {
    if (!grid_ok(g) || !st || !cfg) return OC_ERR_ARG;
    oc::PlanInput in = plan_input(g, st, cfg);
    in.rate = ckpt_rate_bits;
    in.slab_planes = cfg->slab_planes;
    oc::AdjPlan a;
    int r = oc::make_adj_plan(in, ckpt_every, steps, &a);
    if (r != oc::ST_OK) return r;
    std::vector<oc::Op> ops;
    oc::build_adjoint_ops(a, 0, &ops);
    if (mutate == 1) {
      int64_t seen = 0;
      bool dropped = false;
      for (size_t j = 0; j < ops.size(); j++)
        if (ops[j].type == oc::OP_WAIT && seen++ == i) {
          ops.erase(ops.begin() + (ptrdiff_t)j);
          dropped = true;
          break;
        }
      if (!dropped) return OC_ERR_ARG;
    } else if (mutate != 0) {
      return OC_ERR_ARG;
    }
    std::string why;
    int64_t bad = oc::check_ops(a.g, ops, &why);
    if (bad && getenv("OC_CHECK_VERBOSE")) fprintf(stderr, "oc adjoint check: %s\n", why.c_str());
    if (mutate == 0 && i == -1) {
      int64_t w = 0;
      for (const auto &o : ops) w += o.type == oc::OP_WAIT;
      return w;   // number of waits (for the mutation sweep)
    }
    return bad;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_debug_copy_to_host(void *host_base, size_t host_off, const void *dev_src, size_t bytes,
                          int32_t workgroups, oc_stream stream) {
  try {
    if (!host_base || !dev_src || workgroups < 1 || workgroups > 1024) return OC_ERR_ARG;
    uint8_t *dst = mapped_host(host_base);
    if (!dst) return OC_ERR_ARG;   // not pinned, mapped host memory
    hipError_t e = oc::launch_copy_to_host(dst + host_off, dev_src, bytes, workgroups,
                                           (hipStream_t)stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_debug_codec_star7(const void *d_in, void *d_out, int64_t nx, int64_t ny, int64_t nz, int64_t gz0,
                         int64_t out_nl, int64_t lay_lo, int64_t lay_hi, int32_t rate_bits, int32_t steps,
                         const float *c, oc_stream stream) {
  try {
    if (!d_in || !d_out || !c || nx <= 0 || ny <= 0 || nz <= 0 || out_nl < 1) return OC_ERR_ARG;
    if (((uintptr_t)d_in | (uintptr_t)d_out) & 3) return OC_ERR_ARG;
    if (nx % 4 || ny % 4 || nz % 4 || gz0 % 4) return OC_ERR_SHAPE;
    if (rate_bits < 1 || rate_bits > oc::kCodecStar7MaxRate || steps < 1 || steps > 4)
      return OC_ERR_UNSUPPORTED;
    const int64_t nl = out_nl + 2;
    if (lay_lo < 0 || lay_hi > nl || lay_lo > lay_hi) return OC_ERR_ARG;
    // coded layers must lie inside the grid, the interior too
    if (gz0 + 4 * lay_lo < 0 || gz0 + 4 * lay_hi > nz || gz0 + 4 < 0 || gz0 + 4 * (1 + out_nl) > nz)
      return OC_ERR_ARG;
    const oc::Star7Coef cf{c[0], c[1], c[2], c[3], c[4], c[5], c[6]};
    hipError_t e = oc::launch_codec_star7(d_in, d_out, nx, ny, rate_bits, lay_lo, lay_hi, nl, 1, out_nl, gz0,
                                          nz, steps, cf, (hipStream_t)stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_stream_overlap(oc_stream a, oc_stream b, double *overlap) {
  try {
    if (!a || !b || !overlap) return OC_ERR_ARG;
    hipError_t e = oc::probe_stream_overlap((hipStream_t)a, (hipStream_t)b, overlap);
    if (e != hipSuccess) {
      g_last_hip = e;
      return OC_ERR_HIP;
    }
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int64_t oc_debug_timeline(const oc_handle *h, int32_t *kind, int64_t *slab, double *start_ms,
                          double *end_ms, int64_t cap) {
  try {
    if (!h) return OC_ERR_ARG;
    const int64_t n = (int64_t)h->last_timed.size();
    if (!kind || !slab || !start_ms || !end_ms || cap <= 0) return n;
    if (h->broken || n == 0) return n == 0 ? 0 : OC_ERR_STATE;
    const hipEvent_t base = h->tev[h->last_timed[0].ev];
    const int64_t m = std::min(n, cap);
    for (int64_t i = 0; i < m; i++) {
      const auto &t = h->last_timed[(size_t)i];
      float a = 0.f, b = 0.f;
      if (hipEventElapsedTime(&a, base, h->tev[t.ev]) != hipSuccess ||
          hipEventElapsedTime(&b, base, h->tev[t.ev + 1]) != hipSuccess)
        return OC_ERR_HIP;
      kind[i] = t.kind;
      slab[i] = t.slab;
      start_ms[i] = a;
      end_ms[i] = b;
    }
    return m;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_stats_get(const oc_handle *h, oc_stats *s) {
  try {
    if (!h || !s) return OC_ERR_ARG;
    *s = h->stats;
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_set_timing(oc_handle *h, int32_t on) {
  try {
    if (!h) return OC_ERR_ARG;
    h->timing = on != 0;
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_destroy(oc_handle *h) {
  try {
    if (!h) return OC_ERR_ARG;
    drain(h);
    for (auto &e : h->ev)
      if (e) (void)hipEventDestroy(e);
    for (auto &e : h->tev)
      if (e) (void)hipEventDestroy(e);
    delete h;
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_debug_fail_after(oc_handle *h, int64_t n) {
  try {
    if (!h) return OC_ERR_ARG;
    h->fail_after = n >= 1 ? n : -1;
    h->hip_calls = 0;
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int oc_debug_serialize(oc_handle *h, int32_t on) {
  try {
    if (!h) return OC_ERR_ARG;
    h->serialize = on != 0;
    return OC_OK;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int64_t oc_debug_plan_ops(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                          int64_t sweeps, int64_t *n_waits) {
  try {
    if (!grid_ok(g) || !st || !cfg || sweeps < 1) return OC_ERR_ARG;
    oc::Plan p;
    int r = oc::make_plan(plan_input(g, st, cfg), &p);
    if (r != oc::ST_OK) return r;
    std::vector<oc::Op> ops;
    oc::build_ops(p, sweeps, p.in.k, 0, 0, &ops, nullptr, p.load_rate);
    if (n_waits) {
      int64_t w = 0;
      for (const auto &o : ops) w += o.type == oc::OP_WAIT;
      *n_waits = w;
    }
    return (int64_t)ops.size();
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int64_t oc_debug_plan_dump(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                           int64_t sweeps, char *buf, size_t len) {
  try {
    if (!grid_ok(g) || !st || !cfg || sweeps < 1) return OC_ERR_ARG;
    oc::Plan p;
    int r = oc::make_plan(plan_input(g, st, cfg), &p);
    if (r != oc::ST_OK) return r;
    std::vector<oc::Op> ops;
    oc::build_ops(p, sweeps, p.in.k, 0, 0, &ops, nullptr, p.load_rate);
    std::string s = oc::dump_ops(ops);
    if (buf && len) {
      size_t n = std::min(len - 1, s.size());
      std::memcpy(buf, s.data(), n);
      buf[n] = 0;
    }
    return (int64_t)s.size() + 1;
  } catch (...) {
    return OC_ERR_HOST;
  }
}

namespace {

// ckpt_rate < 0: no checkpoint output
int64_t check_plan_impl(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                        int64_t sweeps, int32_t ckpt_rate, int32_t mutate, int64_t i) {
  if (!grid_ok(g) || !st || !cfg || sweeps < 1) return OC_ERR_ARG;
  oc::Plan p;
  int r = oc::make_plan(plan_input(g, st, cfg), &p);
  if (r != oc::ST_OK) return r;
  if (mutate == 4) {  // in place without region sharing: slabs reread updated planes
    if (!p.in_place) return OC_ERR_ARG;
    p.share = false;
  }
  oc::CkptOut ck;
  if (ckpt_rate >= 0) {
    if (ckpt_rate > 32 || !oc::ckpt_out_supported(p, ckpt_rate)) return OC_ERR_UNSUPPORTED;
    ck.rate = ckpt_rate;
  }
  std::vector<oc::Op> ops;
  oc::build_ops(p, sweeps, p.in.k, 0, 0, &ops, ckpt_rate >= 0 ? &ck : nullptr, p.load_rate);
  if (mutate == 0 && i == -1) {   // the number of waits
    int64_t n = 0;
    for (const oc::Op &o : ops) n += o.type == oc::OP_WAIT;
    return n;
  }
  if (mutate == 1) {  // drop the i-th wait
    int64_t seen = 0;
    bool dropped = false;
    for (size_t j = 0; j < ops.size(); j++)
      if (ops[j].type == oc::OP_WAIT && seen++ == i) {
        ops.erase(ops.begin() + (ptrdiff_t)j);
        dropped = true;
        break;
      }
    if (!dropped) return OC_ERR_ARG;
  } else if (mutate == 2) {  // drop the epilogue: everything after the last kernel
    size_t last = 0;
    for (size_t j = 0; j < ops.size(); j++)
      if (ops[j].type == oc::OP_STAR7 || ops[j].type == oc::OP_WAVE || ops[j].type == oc::OP_FUSED) last = j;
    ops.erase(ops.begin() + (ptrdiff_t)last + 1, ops.end() - 1);
  } else if (mutate == 3) {  // swap op i with the next op of the same stream
    if (i < 0 || (size_t)i >= ops.size() || ops[(size_t)i].stream < 0) return OC_ERR_ARG;
    for (size_t j = (size_t)i + 1; j < ops.size(); j++)
      if (ops[j].stream == ops[(size_t)i].stream) {
        std::swap(ops[(size_t)i], ops[j]);
        break;
      }
  } else if (mutate == 5) {  // second sweep copies in from the level the first one read
    if (p.in_place || sweeps < 2) return OC_ERR_ARG;
    for (auto &o : ops)
      if (o.type == oc::OP_H2D && o.sweep == 1 && o.host_id <= oc::HOST_LEVEL1) o.host_id ^= 1;
  } else if (mutate != 0 && mutate != 4) {
    return OC_ERR_ARG;
  }
  std::string why;
  int64_t bad = oc::check_ops(p, ops, &why);
  if (bad && getenv("OC_CHECK_VERBOSE")) fprintf(stderr, "oc plan check: %s\n", why.c_str());
  return bad;
}

}  // namespace

int64_t oc_debug_check_plan(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                            int64_t sweeps, int32_t mutate, int64_t i) {
  try {
    return check_plan_impl(g, st, cfg, sweeps, -1, mutate, i);
  } catch (...) {
    return OC_ERR_HOST;
  }
}

int64_t oc_debug_check_plan_ckpt(const oc_grid *g, const oc_stencil *st, const oc_config *cfg,
                                 int64_t sweeps, int32_t ckpt_rate_bits, int32_t mutate, int64_t i) {
  try {
    if (ckpt_rate_bits < 0) return OC_ERR_ARG;
    return check_plan_impl(g, st, cfg, sweeps, ckpt_rate_bits, mutate, i);
  } catch (...) {
    return OC_ERR_HOST;
  }
}

}  // extern "C"
