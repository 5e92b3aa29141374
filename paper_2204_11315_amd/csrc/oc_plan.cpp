// oc_plan.cpp -- slab planner, arena carve-out, operation list, and the
// happens-before checker over that list.  Host-only C++.
//
// Out-of-core decomposition (Sec. 3.1): the z extent is cut into slabs of S
// interior planes; each residency loads S + 2*halo planes so that k time steps
// can run on the GPU before the slab goes back (temporal blocking, Sec. 3.1 and
// Sec. 3.2: more steps per residency means more halo).  With a coded host
// store the halo is rounded up to whole 4-plane block layers.
//
// Issue order (Sec. 5, Algorithm 1 and Fig. 4): three streams overlap the
// copy-in, the kernels and the copy-back.  Here each stream has one role --
// stream 0 copies in, stream 1 runs every kernel (decode, k stencil steps,
// encode), stream 2 copies back -- and the g-th slab uses slot g mod 3 of a
// ring of three coded staging buffers.  Events link the roles: the slab's
// copy-in done (-> its kernels), "slot coded" (kernels -> copy-back) and the
// slab's copy-back done (-> the next copy-in into that slot).  The copy-in and
// copy-back events are the per-slab ones below, so each copy stream records
// one event per slab: a marker on those streams costs the job ~1.5 % per slab
// (measured).  Because all kernels run on one
// stream, the single shared working buffer (Sec. 5) is ordered by stream
// order alone; the paper's "wait for the cyclically prior stream" edge
// (Fig. 7) becomes that stream order.  Giving each DMA direction its own
// stream keeps a copy-back from queueing in front of an unrelated copy-in.
// The paper updates its host chunks in place, which with temporal-blocking
// halos needs region sharing or separate compression of the overlap
// (Sec. 3.1, Sec. 4.1); instead the host keeps two levels that alternate as
// source and destination by sweep, with per-slab copy events ordering the
// cross-sweep reuse:
//   copy-in of slab j in sweep t waits for the copy-back of every slab of
//   sweep t-1 whose interior it reads (halo overlap), and the copy-back of
//   slab j in sweep t waits for every copy-in of sweep t-1 that read the planes
//   it overwrites.  (One level updated in place, with region sharing, is the
//   alternative: see make_plan.)
// Waits already implied by stream order and earlier waits are left out.
#include "oc_plan.h"

#include <algorithm>
#include <cstdio>

namespace oc {

int stencil_radius(int kind) { return kind == KIND_WAVE25 ? 4 : 1; }

size_t coded_layer_bytes(int64_t nx, int64_t ny, int rate) {
  return (size_t)(nx / 4) * (size_t)(ny / 4) * 8u * (size_t)rate;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves the arena for a given S; returns total bytes.
static size_t carve(Plan *p) {
  const PlanInput &in = p->in;
  p->P = p->S + 2 * p->halo;
  p->work_bytes = align256((size_t)p->P * p->plane_bytes);
  size_t off = 0;
  if (p->fused) {
    // slots of input codes + interior codes; the arena also has to hold the
    // two FP32 chunks of at least 4 planes (and their codes) that oc_load and
    // oc_store stage through it
    p->fused_out = align256((size_t)(p->P / 4) * p->layer_bytes);
    p->stage_bytes = p->fused_out + align256((size_t)(p->S / 4) * p->layer_bytes);
    for (int s = 0; s < p->slots; s++) {
      p->off_stage[s] = off;
      off += p->stage_bytes;
    }
    const size_t io = 2u * align256(4u * p->plane_bytes) + 2u * align256(p->layer_bytes);
    return std::max(off, io);
  }
  for (int s = 0; s < p->n_work_sets; s++)
    for (int b = 0; b < p->n_work_bufs; b++) {
      p->off_work[s][b] = off;
      off += p->work_bytes;
    }
  for (int s = p->n_work_sets; s < kMaxSlots; s++)
    for (int b = 0; b < p->n_work_bufs; b++) p->off_work[s][b] = p->off_work[0][b];
  p->stage_bytes = 0;
  if (p->coded) {
    int fields_in = p->n_rw + (p->ro_coded ? 1 : 0);
    p->stage_bytes = align256((size_t)(p->P / 4) * p->max_layer_bytes * (size_t)fields_in);
    for (int s = 0; s < p->slots; s++) {
      p->off_stage[s] = off;
      off += p->stage_bytes;
    }
  }
  // STAR7 with a raw c0 field in single-buffer mode: the c0 slab is copied in
  // per ring slot (it is read-only, so no copy back), then moved into the
  // shared set on the kernel stream.
  if (in.kind == KIND_STAR7 && in.c0_field && p->n_work_sets == 1) {
    for (int s = 0; s < p->slots; s++) {
      p->off_ro_stage[s] = off;
      off += p->work_bytes;
    }
  }
  // uncompressed 25-point runs with region sharing: a stash per slot for the
  // shared planes of the two pressure fields
  p->stash_bytes = 0;
  if (in.kind == KIND_WAVE25 && !p->coded && in.share) {
    p->stash_bytes = align256(2u * (size_t)(2 * p->halo) * p->plane_bytes);
    for (int s = 0; s < p->slots; s++) {
      p->off_stash[s] = off;
      off += p->stash_bytes;
    }
  }
  (void)in;
  return off;
}

int make_plan(const PlanInput &in, Plan *out) {
  Plan p;
  p.in = in;
  if (in.nx <= 0 || in.ny <= 0 || in.nz <= 0 || in.k < 1 || in.rate < 0 || in.rate > 32 ||
      in.slab_planes < 0 || (in.kind != KIND_STAR7 && in.kind != KIND_WAVE25))
    return ST_ARG;
  // a load rate: coded runs only, at least the rate; the 25-point fields and
  // the fused kernel (one rate in and out) take one rate
  if (in.load_rate < 0 || in.load_rate > 32 || (in.load_rate > 0 && (in.rate == 0 || in.load_rate < in.rate)))
    return ST_ARG;
  // (one host level updated in place would hold codes at both strides at once)
  if (in.load_rate > in.rate && (in.kind != KIND_STAR7 || in.fused_codec || in.in_place))
    return ST_UNSUPPORTED;
  if (in.kind == KIND_WAVE25 && in.c0_field) return ST_ARG;
  if (in.slots < 2 || in.slots > kMaxSlots || in.prefetch >= in.slots) return ST_ARG;
  if (in.fuse < 1 || in.fuse > kMaxFused) return ST_ARG;
  p.slots = in.slots;
  p.prefetch = in.prefetch < 0 ? in.slots - 1 : in.prefetch;
  p.r = stencil_radius(in.kind);
  p.coded = in.rate > 0;
  if (in.fused_codec) {
    // the fused kernel: coded 7-point runs with constant coefficients, up to
    // four steps per residency (one block layer of halo), rates its LDS holds
    if (!p.coded || in.kind != KIND_STAR7 || in.c0_field || in.k > kMaxFused || in.rate > kFusedMaxRate)
      return ST_UNSUPPORTED;
    p.fused = true;
  }
  if (p.coded && (in.nx % 4 || in.ny % 4 || in.nz % 4)) return ST_SHAPE;
  if (p.coded && in.slab_planes % 4) return ST_SHAPE;
  if (in.nx > (int64_t)1 << 30 || in.ny > (int64_t)1 << 30 || in.nz > (int64_t)1 << 30)
    return ST_ARG;
  p.n_rw = in.kind == KIND_WAVE25 ? 2 : 1;
  p.has_ro = in.kind == KIND_WAVE25 || in.c0_field;
  p.ro_coded = p.coded && in.kind == KIND_WAVE25;
  p.plane_bytes = (size_t)in.nx * (size_t)in.ny * 4u;
  p.layer_bytes = p.coded ? coded_layer_bytes(in.nx, in.ny, in.rate) : 0;
  p.load_rate = std::max(in.load_rate, in.rate);
  p.max_layer_bytes = p.coded ? coded_layer_bytes(in.nx, in.ny, p.load_rate) : 0;
  int64_t h = (int64_t)in.k * p.r;
  p.halo = p.coded ? (h + 3) / 4 * 4 : h;
  // working buffers: STAR7 a, b (+ c0 slab); WAVE25 v, pa, pb
  p.n_work_bufs = in.kind == KIND_WAVE25 ? 3 : (in.c0_field ? 3 : 2);
  // uncompressed runs keep one working set per ring slot (three, as the three
  // per-stream buffers of Fig. 5a); compressed runs share one set (Sec. 5)
  // unless asked otherwise (three, Fig. 5b).
  p.n_work_sets = (p.coded && in.single_buffer) ? 1 : p.slots;

  const int64_t step = p.coded ? 4 : 1;
  if (in.slab_planes > 0) {
    p.S = std::min<int64_t>(in.slab_planes, p.coded ? (in.nz + 3) / 4 * 4 : in.nz);
    p.arena_bytes = carve(&p);
    if (in.budget && p.arena_bytes > in.budget) return ST_BUDGET;
  } else {
    // largest S (multiple of `step`, at most nz) whose carve-out fits
    int64_t best = 0;
    int64_t lo = step, hi = (in.nz + step - 1) / step * step;
    while (lo <= hi) {
      int64_t mid = (lo + hi) / 2 / step * step;
      if (mid < lo) mid = lo;
      p.S = mid;
      size_t need = carve(&p);
      if (!in.budget || need <= in.budget) {
        best = mid;
        lo = mid + step;
      } else {
        hi = mid - step;
      }
    }
    if (!best) return ST_BUDGET;
    p.S = best;
    p.arena_bytes = carve(&p);
  }
  // slabs
  for (int64_t z0 = 0; z0 < in.nz; z0 += p.S) {
    Slab s;
    s.z0 = z0;
    s.z1 = std::min<int64_t>(z0 + p.S, in.nz);
    s.gz0 = z0 - p.halo;
    s.l0 = std::max<int64_t>(0, z0 - p.halo);
    s.l1 = std::min<int64_t>(in.nz, s.z1 + p.halo);
    s.planes = (s.z1 - s.z0) + 2 * p.halo;
    p.slabs.push_back(s);
  }
  // host storage
  int64_t cells = in.nx * in.ny * in.nz;
  p.host_field_bytes = p.coded ? (size_t)(in.nz / 4) * p.max_layer_bytes : (size_t)cells * 4u;
  p.host_level_bytes = p.host_field_bytes * (size_t)p.n_rw;
  p.host_aux_bytes = 0;
  if (in.kind == KIND_WAVE25) p.host_aux_bytes = p.host_field_bytes;
  if (in.c0_field) p.host_aux_bytes = (size_t)cells * 4u;
  // region sharing (Sec. 3.1, Fig. 2): consecutive slabs of a sweep both load
  // the 2h planes around their common face; the later one takes them from the
  // earlier one's input on the device.  The earlier input must survive its own
  // kernels: coded inputs live in the staging slot, past the encoder's output;
  // raw inputs survive only when one stencil launch covers all k steps.
  // (the 25-point leapfrog overwrites its raw inputs in place: uncompressed
  // runs set the shared planes aside in a per-slot stash first)
  p.share = in.share && p.slabs.size() >= 2 &&
            ((in.kind == KIND_STAR7 && (p.coded || in.k <= in.fuse)) ||
             (in.kind == KIND_WAVE25 && (p.coded ? p.ro_coded : p.stash_bytes > 0)));
  // one host level updated in place (the Ensure clause of Algorithm 1): a
  // slab's copy-back overwrites its interior planes, which the next slab of
  // the sweep still needs as old values around their common face, so every
  // face must be shared on the device (or there is only one slab)
  if (in.in_place && !(p.share || p.slabs.size() == 1)) return ST_ARG;
  p.in_place = in.in_place;
  *out = p;
  return ST_OK;
}

// ---------------------------------------------------------------------------
// operation list
// ---------------------------------------------------------------------------
namespace {

struct Builder {
  const Plan &p;
  std::vector<Op> *ops;
  EventIds ev;
  // Vector clocks of the streams and of each event's last record, used to
  // leave out waits that stream order and earlier waits already imply.
  int64_t vc[3][3] = {};
  std::vector<std::array<int64_t, 3>> evc;
  Builder(const Plan &pl, std::vector<Op> *o) : p(pl), ops(o) {
    ev.n_slabs = (int)pl.slabs.size();
    evc.assign((size_t)ev.count(), {-1, -1, -1});
  }
  Op blank(OpType t, int stream) {
    Op o{};
    o.type = t;
    o.stream = (int8_t)stream;
    o.host_id = -1;
    o.ev = -1;
    o.dev_src = o.dev_src2 = o.dev_dst = -1;
    o.levels = 1;
    o.rate = 0;
    return o;
  }
  void push(const Op &o) {
    if (o.type == OP_SYNC) {
      for (int q = 0; q < 3; q++) {
        int64_t m = 0;
        for (int s = 0; s < 3; s++) m = std::max(m, vc[s][q]);
        for (int s = 0; s < 3; s++) vc[s][q] = m;
      }
    } else if (o.type != OP_REC && o.type != OP_WAIT) {
      vc[o.stream][o.stream]++;
    }
    ops->push_back(o);
  }
  void rec(int s, int e) {
    Op o = blank(OP_REC, s);
    o.ev = e;
    for (int q = 0; q < 3; q++) evc[(size_t)e][q] = vc[s][q];
    push(o);
  }
  void wait(int s, int e) { wait_all(s, {e}); }
  // Waits for every event of `es`, leaving out those already implied by the
  // stream's clock or by another event of the set.
  void wait_all(int s, const std::vector<int> &es) {
    for (size_t a = 0; a < es.size(); a++) {
      const auto &c = evc[(size_t)es[a]];
      bool implied = true;
      for (int q = 0; q < 3; q++) implied &= c[q] <= vc[s][q];
      for (size_t b = 0; b < es.size() && !implied; b++) {
        if (b == a) continue;
        const auto &d = evc[(size_t)es[b]];
        bool le = true, eq = true;
        for (int q = 0; q < 3; q++) {
          le &= c[q] <= d[q];
          eq &= c[q] == d[q];
        }
        implied = le && (!eq || b < a);   // equal clocks: keep the first
      }
      if (implied) continue;
      Op o = blank(OP_WAIT, s);
      o.ev = es[a];
      push(o);
    }
    for (int e : es)
      for (int q = 0; q < 3; q++) vc[s][q] = std::max(vc[s][q], evc[(size_t)e][q]);
  }
  // indices of slabs whose loaded range intersects [a, b)
  void readers_of(int64_t a, int64_t b, std::vector<int> *out) const {
    out->clear();
    for (size_t j = 0; j < p.slabs.size(); j++)
      if (p.slabs[j].l0 < b && a < p.slabs[j].l1) out->push_back((int)j);
  }
  // indices of slabs whose interior intersects [a, b)
  void writers_of(int64_t a, int64_t b, std::vector<int> *out) const {
    out->clear();
    for (size_t j = 0; j < p.slabs.size(); j++)
      if (p.slabs[j].z0 < b && a < p.slabs[j].z1) out->push_back((int)j);
  }
  size_t work(int set, int b) const { return p.off_work[p.n_work_sets == 1 ? 0 : set][b]; }
};

}  // namespace

bool ckpt_out_supported(const Plan &p, int rate) {
  if (p.in.kind != KIND_STAR7 || p.coded) return false;
  if (rate == 0) return true;
  return p.in.nx % 4 == 0 && p.in.ny % 4 == 0 && p.in.nz % 4 == 0 && p.S % 4 == 0;
}

void build_ops(const Plan &p, int64_t sweeps, int steps_last, int src, int64_t step0,
               std::vector<Op> *ops, const CkptOut *ck, int rate0) {
  if (ck && !ckpt_out_supported(p, ck->rate)) ck = nullptr;
  // the first sweep reads codes at rate0 (the loaded codes), later sweeps at
  // the plan's rate; coded layers keep their positions, at each rate's stride
  const int in_rate0 = (p.coded && rate0 > 0) ? rate0 : p.in.rate;
  auto rate_in = [&](int t) { return t == 0 ? in_rate0 : p.in.rate; };
  auto lb_in = [&](int t) {
    return rate_in(t) == p.in.rate ? p.layer_bytes : coded_layer_bytes(p.in.nx, p.in.ny, rate_in(t));
  };
  ops->clear();
  Builder B(p, ops);
  const int ns = (int)p.slabs.size();
  const int64_t total = sweeps * ns;
  const bool swb = p.n_work_sets == 1;
  const bool wave = p.in.kind == KIND_WAVE25;
  const int NQ = p.slots;
  std::vector<int> nb;
  // buffer roles: STAR7 a=0, b=1, c0=2; WAVE25 v=0, pa=1 (p^{n-1}), pb=2 (p^n)
  const int bv = 0, bpa = 1, bpb = 2;

  struct Geo {
    int t, j, q, srcl, dstl, ks;
    int64_t loc0, nload, nz_int;
    const Slab *sl;
    int64_t sh;       // planes taken from the previous slab's input (region sharing)
    int pq;           // previous slab's slot
    int64_t sh_src;   // local plane of the shared planes in the previous slab's buffer
    int64_t pv_planes;   // the previous slab's buffer planes (its field stride in the slot)
  };
  auto geo = [&](int64_t g) {
    Geo x;
    x.t = (int)(g / ns);
    x.j = (int)(g % ns);
    x.q = (int)(g % NQ);
    x.sl = &p.slabs[x.j];
    x.srcl = p.in_place ? 0 : (src + x.t) & 1;
    x.dstl = p.in_place ? 0 : (src + x.t + 1) & 1;
    x.ks = (x.t == sweeps - 1) ? steps_last : p.in.k;
    x.loc0 = x.sl->l0 - x.sl->gz0;   // local plane of the first loaded plane
    x.nload = x.sl->l1 - x.sl->l0;
    x.nz_int = x.sl->z1 - x.sl->z0;
    x.pq = (int)((g + NQ - 1) % NQ);
    x.sh = 0;
    x.sh_src = 0;
    x.pv_planes = 0;
    if (p.share && x.j > 0) {
      const Slab &pv = p.slabs[(size_t)x.j - 1];
      x.sh = std::max<int64_t>(0, std::min(pv.l1, x.sl->l1) - x.sl->l0);
      x.sh_src = x.sl->l0 - pv.gz0;
      x.pv_planes = pv.planes;
    }
    return x;
  };
  // slab g's slot is next written by the copy-in of slab g + NQ; the shared
  // planes of slab g are read by slab g + 1's overlap copy
  auto has_share_copy = [&](int64_t g) { return p.share && g >= 0 && g < total && g % ns != 0; };
  // region sharing, coded fields with the three-kernel path: slab g's decoder
  // reads the shared layers where slab g - 1's copy-in left them (that slab's
  // slot, at the field's stride), so no copy precedes it -- unless slab g + 1
  // shares planes that slab g itself got from slab g - 1 (slabs thinner than
  // the shared region): those must then be in slab g's slot, so they are
  // copied there.  The copy-in that next overwrites slab g - 1's slot then
  // waits for slab g's whole kernel sequence (its "out" event), which the
  // decode precedes, instead of a separate event after the decode.
  auto reads_in_place = [&](int64_t g) {
    if (!p.coded || p.fused || !has_share_copy(g)) return false;
    const Geo x = geo(g);
    if (x.sh <= 0) return false;
    if (has_share_copy(g + 1)) {
      const Geo nx1 = geo(g + 1);
      if (nx1.sh > 0 && nx1.sh_src < x.loc0 + x.sh) return false;
    }
    return true;
  };
  // fields copied in: (host store, base offset, working buffer, coded?)
  struct In { int host_id; size_t host_base; int buf; bool coded; };
  auto inputs = [&](const Geo &x, In *fin) {
    int nin = 0;
    if (wave) {
      fin[nin++] = {x.srcl, 0, bpb, p.coded};                   // p^n
      fin[nin++] = {x.srcl, p.host_field_bytes, bpa, p.coded};  // p^{n-1}
      fin[nin++] = {HOST_AUX, 0, bv, p.ro_coded};               // velocity
    } else {
      fin[nin++] = {x.srcl, 0, 0, p.coded};
      if (p.in.c0_field) fin[nin++] = {HOST_AUX, 0, 2, false};
    }
    return nin;
  };
  const bool c0_staged = swb && !wave && p.in.c0_field;  // raw c0 rides in a per-slot stage
  // inputs region sharing covers: the coded fields, the raw 7-point field and
  // the 7-point c0 field (read-only, so it survives the slab's kernels)
  auto shared_in = [&](const In &fi, int f) {
    return fi.coded || (!p.coded && (f == 0 || wave)) || (!wave && fi.buf == 2);
  };
  // uncompressed 25-point: where slot q's stash keeps the shared planes of a
  // pressure field (p^n first, then p^{n-1})
  auto stash_of = [&](int q, int buf) {
    return p.off_stash[q] + (buf == bpb ? 0u : (size_t)(2 * p.halo) * p.plane_bytes);
  };
  const bool stash = wave && !p.coded && p.share;
  // where a slot keeps its raw c0 slab as loaded
  auto c0_buf = [&](int q) { return c0_staged ? p.off_ro_stage[q] : B.work(q, 2); };

  // ---- copy-in stream: slab g into slot g mod NQ -----------------------------
  auto issue_in = [&](int64_t g) {
    const Geo x = geo(g);
    In fin[3];
    const int nin = inputs(x, fin);
    std::vector<int> w;
    if (g >= NQ) {   // the slot's previous copy-back done (its per-slab copy event)
      const Geo pg = geo(g - NQ);
      w.push_back(B.ev.d2h(pg.t & 1, pg.j));
    }
    if (g >= NQ && has_share_copy(g - NQ + 1)) {
      // the slot's previous slab passed planes on to the next slab; wait for
      // that copy if this copy-in overwrites any of them
      const Geo nx1 = geo(g - NQ + 1);
      const int64_t wlo = x.loc0 + x.sh, whi = x.loc0 + x.nload;
      if (wlo < whi && wlo < nx1.sh_src + nx1.sh && nx1.sh_src < whi)
        w.push_back(reads_in_place(g - NQ + 1) ? B.ev.out(nx1.q) : B.ev.shr(x.q));
    }
    if (x.t > 0) {                                   // planes written by last sweep's copy-backs
      B.writers_of(x.sl->l0, x.sl->l1, &nb);
      for (int jj : nb) w.push_back(B.ev.d2h((x.t - 1) & 1, jj));
    }
    B.wait_all(S_IN, w);
    int ncoded = 0;
    for (int f = 0; f < nin; f++) {
      Op o = B.blank(OP_H2D, S_IN);
      o.host_id = (int8_t)fin[f].host_id;
      // shared inputs skip the planes the overlap copy brings
      const int64_t skip = shared_in(fin[f], f) ? x.sh : 0;
      if (fin[f].coded) {
        // staging slot: layer of local plane z at position z / 4, so the
        // planes shared with the next slab lie past the encoder's output
        const size_t lb = lb_in(x.t);
        o.dev_dst = (int64_t)(p.off_stage[x.q] + (size_t)ncoded * (size_t)(x.sl->planes / 4) * lb +
                              (size_t)((x.loc0 + skip) / 4) * lb);
        o.host_off = (int64_t)(fin[f].host_base + (size_t)((x.sl->l0 + skip) / 4) * lb);
        o.bytes = (int64_t)((size_t)((x.nload - skip) / 4) * lb);
        ncoded++;
      } else if (c0_staged && fin[f].buf == 2) {
        o.dev_dst = (int64_t)(p.off_ro_stage[x.q] + (size_t)(x.loc0 + skip) * p.plane_bytes);
        o.host_off = (int64_t)((size_t)(x.sl->l0 + skip) * p.plane_bytes);
        o.bytes = (int64_t)((size_t)(x.nload - skip) * p.plane_bytes);
      } else {
        o.dev_dst = (int64_t)(B.work(x.q, fin[f].buf) + (size_t)(x.loc0 + skip) * p.plane_bytes);
        o.host_off = (int64_t)(fin[f].host_base + (size_t)(x.sl->l0 + skip) * p.plane_bytes);
        o.bytes = (int64_t)((size_t)(x.nload - skip) * p.plane_bytes);
      }
      o.slab = x.j;
      o.sweep = x.t;
      if (o.bytes > 0) B.push(o);
    }
    B.rec(S_IN, B.ev.h2d(x.t & 1, x.j));
  };

  // ---- kernel stream: decode, k steps, encode -------------------------------
  // returns the working buffers holding the results (STAR7 u; WAVE25 p^n, p^{n-1})
  auto issue_compute = [&](int64_t g, int *res) {
    const Geo x = geo(g);
    In fin[3];
    const int nin = inputs(x, fin);
    B.wait(S_COMPUTE, B.ev.h2d(x.t & 1, x.j));
    // coded shared layers read where the previous slab left them, or moved
    int64_t sh_off[3] = {-1, -1, -1}, sh_bytes[3] = {0, 0, 0};
    const bool read_in_place = reads_in_place(g);
    if (x.sh > 0) {
      // region sharing: the planes around the common face come from the
      // previous slab's input -- coded fields read in place by the decoder
      // (above), otherwise device-to-device moves (raw marker z_hi < 0): a
      // coded field at its stride in the staging slot (fused codec kernel,
      // or planes the next slab needs), the raw field, the raw c0 slab
      int nsh = 0;
      for (int f = 0; f < nin; f++) {
        if (!shared_in(fin[f], f)) continue;
        Op o = B.blank(OP_DEC, S_COMPUTE);
        if (fin[f].coded) {
          const size_t lb = lb_in(x.t);   // the previous slab is of the same sweep
          const int64_t from = (int64_t)(p.off_stage[x.pq] + (size_t)nsh * (size_t)(x.pv_planes / 4) * lb +
                                         (size_t)(x.sh_src / 4) * lb);
          const int64_t nbytes = (int64_t)((size_t)(x.sh / 4) * lb);
          if (read_in_place) {
            sh_off[nsh] = from;
            sh_bytes[nsh] = nbytes;
            nsh++;
            continue;
          }
          // a device-to-device move into this slab's slot
          o.dev_src = from;
          o.dev_dst = (int64_t)(p.off_stage[x.q] + (size_t)nsh * (size_t)(x.sl->planes / 4) * lb +
                                (size_t)(x.loc0 / 4) * lb);
          o.bytes = nbytes;
          nsh++;
        } else if (stash && fin[f].buf != bv) {
          // a pressure field of an uncompressed wave run: from the stash
          o.dev_src = (int64_t)stash_of(x.pq, fin[f].buf);
          o.dev_dst = (int64_t)(B.work(x.q, fin[f].buf) + (size_t)x.loc0 * p.plane_bytes);
          o.bytes = (int64_t)((size_t)x.sh * p.plane_bytes);
        } else {
          const bool c0 = !wave && fin[f].buf == 2;
          const size_t src = c0 ? c0_buf(x.pq) : B.work(x.pq, fin[f].buf);
          const size_t dst = c0 ? c0_buf(x.q) : B.work(x.q, fin[f].buf);
          o.dev_src = (int64_t)(src + (size_t)x.sh_src * p.plane_bytes);
          o.dev_dst = (int64_t)(dst + (size_t)x.loc0 * p.plane_bytes);
          o.bytes = (int64_t)((size_t)x.sh * p.plane_bytes);
        }
        o.z_hi = -1;
        o.planes = x.sh;
        o.slab = x.j;
        o.sweep = x.t;
        B.push(o);
      }
      // the previous slot's shared planes are consumed once the moves are
      // done (when the decodes read them there, the slab's "out" event marks it)
      if (!read_in_place) B.rec(S_COMPUTE, B.ev.shr(x.pq));
    }
    if (p.fused) {
      // one kernel: the slot's codes in, the interior's codes out past them
      Op o = B.blank(OP_FUSED, S_COMPUTE);
      o.dev_src = (int64_t)p.off_stage[x.q];
      o.dev_dst = (int64_t)(p.off_stage[x.q] + p.fused_out);
      o.z_lo = x.loc0 / 4;
      o.z_hi = (x.loc0 + x.nload) / 4;
      o.bytes = (int64_t)((size_t)(x.nz_int / 4) * p.layer_bytes);
      o.levels = x.ks;
      o.gz0 = x.sl->gz0;
      o.planes = x.sl->planes;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
      res[0] = res[1] = 0;
      B.rec(S_COMPUTE, B.ev.out(x.q));
      return;
    }
    int ncoded = 0;
    for (int f = 0; f < nin; f++) {
      if (fin[f].coded) {
        Op o = B.blank(OP_DEC, S_COMPUTE);
        const size_t lb = lb_in(x.t);
        if (rate_in(x.t) != p.in.rate) o.rate = rate_in(x.t);
        o.dev_src = (int64_t)(p.off_stage[x.q] + (size_t)ncoded * (size_t)(x.sl->planes / 4) * lb +
                              (size_t)(x.loc0 / 4) * lb);
        o.dev_dst = (int64_t)(B.work(x.q, fin[f].buf) + (size_t)x.loc0 * p.plane_bytes);
        o.dev_src2 = sh_off[ncoded];
        o.bytes = sh_bytes[ncoded];
        o.z_hi = x.nload / 4;
        o.planes = x.nload;
        o.slab = x.j;
        o.sweep = x.t;
        B.push(o);
        ncoded++;
      } else if (c0_staged && fin[f].buf == 2) {
        Op o = B.blank(OP_DEC, S_COMPUTE);   // device-to-device move (raw marker z_hi < 0)
        o.dev_src = (int64_t)(p.off_ro_stage[x.q] + (size_t)x.loc0 * p.plane_bytes);
        o.dev_dst = (int64_t)(B.work(x.q, 2) + (size_t)x.loc0 * p.plane_bytes);
        o.z_hi = -1;
        o.planes = x.nload;
        o.bytes = (int64_t)((size_t)x.nload * p.plane_bytes);
        o.slab = x.j;
        o.sweep = x.t;
        B.push(o);
      }
    }
    if (stash && has_share_copy(g + 1)) {
      // set the planes the next slab shares aside before the leapfrog
      // overwrites them
      const Geo nx1 = geo(g + 1);
      for (int buf : {bpb, bpa}) {
        if (nx1.sh <= 0) break;
        Op o = B.blank(OP_DEC, S_COMPUTE);
        o.dev_src = (int64_t)(B.work(x.q, buf) + (size_t)nx1.sh_src * p.plane_bytes);
        o.dev_dst = (int64_t)stash_of(x.q, buf);
        o.bytes = (int64_t)((size_t)nx1.sh * p.plane_bytes);
        o.z_hi = -1;
        o.planes = nx1.sh;
        o.slab = x.j;
        o.sweep = x.t;
        B.push(o);
      }
    }
    const int64_t dom_lo = std::max<int64_t>(0, -x.sl->gz0);
    const int64_t dom_hi = std::min<int64_t>(x.sl->planes, p.in.nz - x.sl->gz0);
    int cur_a = 0, cur_b = 1;   // STAR7 ping-pong
    int wa = bpa, wb = bpb;     // WAVE25: wa holds p^{n-1}, wb holds p^n
    // STAR7: the k steps go in groups of up to kMaxFused fused steps; a group
    // ending after step s1 writes its last level on the planes the remaining
    // k - s1 steps still need
    const int group = wave ? 1 : p.in.fuse;
    for (int s0 = 0; s0 < x.ks; s0 += group) {
      const int s1 = std::min(x.ks, s0 + group);
      const int64_t grow = (int64_t)(x.ks - s1) * p.r;
      Op o = B.blank(wave ? OP_WAVE : OP_STAR7, S_COMPUTE);
      if (wave) {
        o.dev_src = (int64_t)B.work(x.q, wb);     // p^n
        o.dev_dst = (int64_t)B.work(x.q, wa);     // p^{n-1} -> p^{n+1}
        o.dev_src2 = (int64_t)B.work(x.q, bv);    // velocity
        o.step = step0 + (int64_t)x.t * p.in.k + s0;
        std::swap(wa, wb);
      } else {
        o.dev_src = (int64_t)B.work(x.q, cur_a);
        o.dev_dst = (int64_t)B.work(x.q, cur_b);
        o.dev_src2 = p.in.c0_field ? (int64_t)B.work(x.q, 2) : -1;
        o.levels = s1 - s0;
        std::swap(cur_a, cur_b);
      }
      o.z_lo = std::max<int64_t>(p.halo - grow, dom_lo);
      o.z_hi = std::min<int64_t>(p.halo + x.nz_int + grow, dom_hi);
      o.gz0 = x.sl->gz0;
      o.planes = x.sl->planes;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    }
    res[0] = wave ? wb : cur_a;
    res[1] = wave ? wa : cur_a;
    if (p.coded) {
      for (int f = 0; f < p.n_rw; f++) {
        Op o = B.blank(OP_ENC, S_COMPUTE);
        o.dev_src = (int64_t)(B.work(x.q, res[f]) + (size_t)p.halo * p.plane_bytes);
        // field f at its input stride, so the shared layers past each
        // field's output survive for the next slab
        o.dev_dst = (int64_t)(p.off_stage[x.q] + (size_t)f * (size_t)(x.sl->planes / 4) * p.layer_bytes);
        o.z_hi = x.nz_int / 4;
        o.planes = x.nz_int;
        o.slab = x.j;
        o.sweep = x.t;
        B.push(o);
      }
    }
    if (ck && ck->rate > 0 && x.t == sweeps - 1) {
      // checkpoint codes of the new state, written into the slot's other
      // working buffer from its first plane on: they end at or below plane S,
      // under the planes the next slab may share
      Op o = B.blank(OP_ENC, S_COMPUTE);
      o.rate = ck->rate;
      o.dev_src = (int64_t)(B.work(x.q, res[0]) + (size_t)p.halo * p.plane_bytes);
      o.dev_dst = (int64_t)B.work(x.q, 1 - res[0]);
      o.z_hi = x.nz_int / 4;
      o.planes = x.nz_int;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    }
    B.rec(S_COMPUTE, B.ev.out(x.q));
  };

  // ---- copy-back stream ---------------------------------------------------------
  auto issue_out = [&](int64_t g, const int *res) {
    const Geo x = geo(g);
    std::vector<int> w{B.ev.out(x.q)};
    if (x.t > 0) {   // planes read by last sweep's copy-ins of this level
      B.readers_of(x.sl->z0, x.sl->z1, &nb);
      for (int jj : nb) w.push_back(B.ev.h2d((x.t - 1) & 1, jj));
    }
    B.wait_all(S_OUT, w);
    for (int f = 0; f < p.n_rw; f++) {
      Op o = B.blank(OP_D2H, S_OUT);
      o.host_id = (int8_t)x.dstl;
      if (p.fused) {
        o.dev_src = (int64_t)(p.off_stage[x.q] + p.fused_out);
        o.host_off = (int64_t)((size_t)(x.sl->z0 / 4) * p.layer_bytes);
        o.bytes = (int64_t)((size_t)(x.nz_int / 4) * p.layer_bytes);
      } else if (p.coded) {
        o.dev_src = (int64_t)(p.off_stage[x.q] + (size_t)f * (size_t)(x.sl->planes / 4) * p.layer_bytes);
        o.host_off = (int64_t)((size_t)f * p.host_field_bytes + (size_t)(x.sl->z0 / 4) * p.layer_bytes);
        o.bytes = (int64_t)((size_t)(x.nz_int / 4) * p.layer_bytes);
      } else {
        o.dev_src = (int64_t)(B.work(x.q, res[f]) + (size_t)p.halo * p.plane_bytes);
        o.host_off = (int64_t)((size_t)f * p.host_field_bytes + (size_t)x.sl->z0 * p.plane_bytes);
        o.bytes = (int64_t)((size_t)x.nz_int * p.plane_bytes);
      }
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    }
    if (ck && x.t == sweeps - 1) {   // the checkpoint copy of the slab's interior
      Op o = B.blank(OP_D2H, S_OUT);
      o.host_id = (int8_t)HOST_CKPT;
      if (ck->rate > 0) {
        const size_t lb = coded_layer_bytes(p.in.nx, p.in.ny, ck->rate);
        o.dev_src = (int64_t)B.work(x.q, 1 - res[0]);
        o.host_off = (int64_t)(ck->host_off + (size_t)(x.sl->z0 / 4) * lb);
        o.bytes = (int64_t)((size_t)(x.nz_int / 4) * lb);
      } else {
        o.dev_src = (int64_t)(B.work(x.q, res[0]) + (size_t)p.halo * p.plane_bytes);
        o.host_off = (int64_t)(ck->host_off + (size_t)x.sl->z0 * p.plane_bytes);
        o.bytes = (int64_t)((size_t)x.nz_int * p.plane_bytes);
      }
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    }
    B.rec(S_OUT, B.ev.d2h(x.t & 1, x.j));
  };

  // Copy-ins run up to `prefetch` slabs ahead and are issued before the
  // copy-back of the slab being computed, so a copy-back that still waits for
  // its kernels never sits in front of a copy-in that could already run.  A
  // copy-in of sweep t is issued only after the copy-backs of sweep t-1 it
  // depends on have been issued (with few slabs per sweep that limits the
  // look-ahead), since a wait can only name an event already recorded.
  const int L = p.prefetch;
  int64_t next_in = 0, outs_issued = 0, computes_issued = 0;
  auto in_ready = [&](int64_t gi) {
    // with region sharing, the copy-in that reuses a slot waits for the
    // overlap copy of the slab after the slot's previous one
    if (gi >= NQ && has_share_copy(gi - NQ + 1) && gi - NQ + 1 >= computes_issued) {
      const Geo xi = geo(gi), nx1 = geo(gi - NQ + 1);
      const int64_t wlo = xi.loc0 + xi.sh, whi = xi.loc0 + xi.nload;
      if (wlo < whi && wlo < nx1.sh_src + nx1.sh && nx1.sh_src < whi) return false;
    }
    const int t = (int)(gi / ns);
    if (t == 0) return true;
    const Slab &sl = p.slabs[(size_t)(gi % ns)];
    B.writers_of(sl.l0, sl.l1, &nb);
    int jmax = 0;
    for (int jj : nb) jmax = std::max(jmax, jj);
    return (int64_t)(t - 1) * ns + jmax < outs_issued;
  };
  for (int64_t g = 0; g < total; g++) {
    while (next_in < total && next_in <= g + L && in_ready(next_in)) issue_in(next_in++);
    int res[2];
    issue_compute(g, res);
    computes_issued = g + 1;
    issue_out(g, res);
    outs_issued = g + 1;
  }
  B.push(B.blank(OP_SYNC, -1));
}

// ---------------------------------------------------------------------------
// adjoint plan and reverse-sweep operation list
// ---------------------------------------------------------------------------
int make_adj_plan(const PlanInput &in0, int m, int64_t steps, AdjPlan *out) {
  if (m < 1 || steps < 1 || in0.kind != KIND_STAR7) return ST_ARG;
  PlanInput in = in0;
  in.slots = 2;        // two full working sets: the copy-in of the next slab
  in.prefetch = 1;     // overlaps the kernels of the current one
  in.load_rate = 0;    // the reverse sweeps read checkpoints at their own rate
  AdjPlan a;
  a.m = m;
  a.steps = steps;
  a.nseg = (int)((steps + m - 1) / m);
  a.ckpt_rate = in.rate;
  Plan &p = a.g;
  p.in = in;
  if (in.nx <= 0 || in.ny <= 0 || in.nz <= 0 || in.rate < 0 || in.rate > 32) return ST_ARG;
  p.r = 1;
  p.coded = in.rate > 0;
  if (p.coded && (in.nx % 4 || in.ny % 4 || in.nz % 4 || in.slab_planes % 4)) return ST_SHAPE;
  p.slots = 2;
  p.prefetch = 1;
  p.n_rw = 1;
  p.plane_bytes = (size_t)in.nx * (size_t)in.ny * 4u;
  p.layer_bytes = p.coded ? coded_layer_bytes(in.nx, in.ny, in.rate) : 0;
  p.load_rate = in.rate;
  p.max_layer_bytes = p.layer_bytes;
  p.halo = p.coded ? ((int64_t)m + 3) / 4 * 4 : m;
  p.n_work_sets = 2;
  p.n_work_bufs = 7;
  auto carve_adj = [&](int64_t S) {
    p.S = S;
    p.P = S + 2 * p.halo;
    p.work_bytes = align256((size_t)p.P * p.plane_bytes);
    p.stage_bytes = p.coded ? align256((size_t)(p.P / 4) * p.layer_bytes) : 0;
    size_t off = 0;
    for (int q = 0; q < 2; q++) {
      for (int b : {A_U0, A_LA, A_LB, A_LC, A_C, A_G}) {
        a.off_buf[q][b] = off;
        off += p.work_bytes;
      }
      a.off_cstage[q] = off;
      off += p.stage_bytes;
    }
    for (int b : {A_WA, A_WB}) {   // only kernels touch them: one pair serves both slots
      a.off_buf[0][b] = a.off_buf[1][b] = off;
      off += p.work_bytes;
    }
    return off;
  };
  const int64_t step = p.coded ? 4 : 1;
  int64_t S = 0;
  if (in.slab_planes > 0) {
    S = std::min<int64_t>(in.slab_planes, (in.nz + step - 1) / step * step);
    if (in.budget && carve_adj(S) > in.budget) return ST_BUDGET;
  } else {
    for (int64_t s = (in.nz + step - 1) / step * step; s >= step; s -= step)
      if (!in.budget || carve_adj(s) <= in.budget) {
        S = s;
        break;
      }
    if (!S) return ST_BUDGET;
  }
  p.arena_bytes = carve_adj(S);
  for (int64_t z0 = 0; z0 < in.nz; z0 += p.S) {
    Slab sl;
    sl.z0 = z0;
    sl.z1 = std::min<int64_t>(z0 + p.S, in.nz);
    sl.gz0 = z0 - p.halo;
    sl.l0 = std::max<int64_t>(0, z0 - p.halo);
    sl.l1 = std::min<int64_t>(in.nz, sl.z1 + p.halo);
    sl.planes = (sl.z1 - sl.z0) + 2 * p.halo;
    p.slabs.push_back(sl);
  }
  p.share = in.share && p.slabs.size() >= 2;
  a.field_bytes = (size_t)in.nx * (size_t)in.ny * (size_t)in.nz * 4u;
  p.host_field_bytes = a.field_bytes;
  p.host_level_bytes = a.field_bytes;   // lambda levels and the gradient store: raw fields
  p.host_aux_bytes = in.c0_field ? a.field_bytes : 0;
  size_t off = 0;
  for (int sg = 0; sg < a.nseg; sg++) {
    a.ckpt_off.push_back(off);
    const int coded = (p.coded && sg > 0) ? 1 : 0;   // the start state stays exact
    a.ckpt_coded.push_back(coded);
    off += coded ? (size_t)(in.nz / 4) * p.layer_bytes : a.field_bytes;
  }
  a.ckpt_bytes = off;
  *out = a;
  return ST_OK;
}

void build_adjoint_ops(const AdjPlan &a, int lsrc, std::vector<Op> *ops) {
  ops->clear();
  const Plan &p = a.g;
  Builder B(p, ops);
  const int ns = (int)p.slabs.size();
  const int64_t total = (int64_t)a.nseg * ns;
  const int NQ = 2;
  const bool c0f = p.in.c0_field;
  std::vector<int> nb;
  struct Geo {
    int t, sg, j, q, lsrc, ldst;
    int64_t n0, len, loc0, nload, nz_int;
    const Slab *sl;
    int pq;           // previous slab's slot
    int64_t sh;       // planes taken from the previous slab's buffers (region sharing)
    int64_t sh_src;   // their local position in the previous slab's buffers
  };
  auto geo = [&](int64_t g) {
    Geo x;
    x.t = (int)(g / ns);
    x.sg = a.nseg - 1 - x.t;                 // segments run newest first
    x.j = (int)(g % ns);
    x.q = (int)(g % NQ);
    x.sl = &p.slabs[x.j];
    x.lsrc = (lsrc + x.t) & 1;
    x.ldst = (lsrc + x.t + 1) & 1;
    x.n0 = (int64_t)x.sg * a.m;
    x.len = std::min<int64_t>(a.m, a.steps - x.n0);
    x.loc0 = x.sl->l0 - x.sl->gz0;
    x.nload = x.sl->l1 - x.sl->l0;
    x.nz_int = x.sl->z1 - x.sl->z0;
    x.pq = (int)((g + NQ - 1) % NQ);
    x.sh = 0;
    x.sh_src = 0;
    if (p.share && x.j > 0) {
      const Slab &pv = p.slabs[(size_t)x.j - 1];
      x.sh = std::max<int64_t>(0, std::min(pv.l1, x.sl->l1) - x.sl->l0);
      x.sh_src = x.sl->l0 - pv.gz0;
    }
    return x;
  };
  // slab g copies planes out of slab g-1's slot at the start of its kernels
  auto has_share_copy = [&](int64_t g) { return p.share && g >= 0 && g < total && g % ns != 0; };
  const size_t pb = p.plane_bytes;
  auto buf = [&](int q, int b) { return (int64_t)a.off_buf[q][b]; };
  auto h2d = [&](const Geo &x, int host, size_t host_off, int64_t dev, int64_t bytes) {
    if (bytes <= 0) return;
    Op o = B.blank(OP_H2D, S_IN);
    o.host_id = (int8_t)host;
    o.host_off = (int64_t)host_off;
    o.dev_dst = dev;
    o.bytes = bytes;
    o.slab = x.j;
    o.sweep = x.t;
    B.push(o);
  };
  auto issue_in = [&](int64_t g) {
    const Geo x = geo(g);
    std::vector<int> w;
    if (g >= NQ) w.push_back(B.ev.free(x.q));
    if (g >= NQ && has_share_copy(g - NQ + 1)) {
      // the next slab of this slot's previous slab copies planes out of the
      // slot; wait for that copy if this copy-in overwrites any of them
      const Geo n1 = geo(g - NQ + 1);
      const int64_t wlo = x.loc0 + x.sh, whi = x.loc0 + x.nload;
      if (wlo < whi && wlo < n1.sh_src + n1.sh && n1.sh_src < whi) w.push_back(B.ev.shr(x.q));
    }
    if (x.t > 0) {
      B.writers_of(x.sl->l0, x.sl->l1, &nb);
      for (int jj : nb) w.push_back(B.ev.d2h((x.t - 1) & 1, jj));
    }
    B.wait_all(S_IN, w);
    // the state, lambda and c0 planes past the shared ones (the gradient
    // store: the interior only)
    const int64_t skip = x.sh;
    if (a.ckpt_coded[(size_t)x.sg])
      h2d(x, HOST_CKPT, a.ckpt_off[(size_t)x.sg] + (size_t)((x.sl->l0 + skip) / 4) * p.layer_bytes,
          (int64_t)(a.off_cstage[x.q] + (size_t)(skip / 4) * p.layer_bytes),
          (int64_t)((size_t)((x.nload - skip) / 4) * p.layer_bytes));
    else
      h2d(x, HOST_CKPT, a.ckpt_off[(size_t)x.sg] + (size_t)(x.sl->l0 + skip) * pb,
          buf(x.q, A_U0) + (x.loc0 + skip) * (int64_t)pb, (x.nload - skip) * (int64_t)pb);
    h2d(x, x.lsrc, (size_t)(x.sl->l0 + skip) * pb, buf(x.q, A_LA) + (x.loc0 + skip) * (int64_t)pb,
        (x.nload - skip) * (int64_t)pb);
    if (c0f)
      h2d(x, HOST_AUX, (size_t)(x.sl->l0 + skip) * pb, buf(x.q, A_C) + (x.loc0 + skip) * (int64_t)pb,
          (x.nload - skip) * (int64_t)pb);
    if (x.t == 0) {
      // the gradient starts at zero: clear the slab's accumulator instead of
      // copying zeros in (the first reverse sweep writes the whole store)
      Op o = B.blank(OP_ZERO, S_IN);
      o.dev_dst = buf(x.q, A_G) + p.halo * (int64_t)pb;
      o.bytes = x.nz_int * (int64_t)pb;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    } else {
      h2d(x, HOST_GRAD, (size_t)x.sl->z0 * pb, buf(x.q, A_G) + p.halo * (int64_t)pb, x.nz_int * (int64_t)pb);
    }
    B.rec(S_IN, B.ev.in(x.q));
    B.rec(S_IN, B.ev.h2d(x.t & 1, x.j));
  };
  auto issue_compute = [&](int64_t g) {
    const Geo x = geo(g);
    B.wait(S_COMPUTE, B.ev.in(x.q));
    if (x.sh > 0) {
      // region sharing: the decoded state, lambda_{n1} and c0 around the
      // common face come from the previous slab's buffers (device moves)
      for (int b : {A_U0, A_LA, A_C}) {
        if (b == A_C && !c0f) continue;
        Op o = B.blank(OP_DEC, S_COMPUTE);
        o.dev_src = buf(x.pq, b) + x.sh_src * (int64_t)pb;
        o.dev_dst = buf(x.q, b) + x.loc0 * (int64_t)pb;
        o.bytes = x.sh * (int64_t)pb;
        o.z_lo = 0;
        o.z_hi = -1;   // raw move
        o.slab = x.j;
        o.sweep = x.t;
        B.push(o);
      }
      B.rec(S_COMPUTE, B.ev.shr(x.pq));
    }
    if (a.ckpt_coded[(size_t)x.sg] && x.nload > x.sh) {
      Op o = B.blank(OP_DEC, S_COMPUTE);
      o.dev_src = (int64_t)(a.off_cstage[x.q] + (size_t)(x.sh / 4) * p.layer_bytes);
      o.dev_dst = buf(x.q, A_U0) + (x.loc0 + x.sh) * (int64_t)pb;
      o.z_hi = (x.nload - x.sh) / 4;
      o.planes = x.nload - x.sh;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    }
    const int64_t dom_lo = std::max<int64_t>(0, -x.sl->gz0);
    const int64_t dom_hi = std::min<int64_t>(x.sl->planes, p.in.nz - x.sl->gz0);
    // `lv` steps (fused in one launch when lv > 1); the output range is the
    // interior grown by `grow` planes per side, clipped to the grid
    auto step = [&](int64_t src, int64_t dst, int64_t grow, bool tr, int lv) {
      Op o = B.blank(OP_STAR7, S_COMPUTE);
      o.dev_src = src;
      o.dev_dst = dst;
      o.dev_src2 = c0f ? buf(x.q, A_C) : -1;
      o.transpose = tr;
      o.levels = lv;
      o.z_lo = std::max<int64_t>(p.halo - grow, dom_lo);
      o.z_hi = std::min<int64_t>(p.halo + x.nz_int + grow, dom_hi);
      o.gz0 = x.sl->gz0;
      o.planes = x.sl->planes;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    };
    const int fuse = std::max(1, std::min(p.in.fuse, kMaxFused));
    // lambda_{n1} stays in La (the next slab may share it); the steps back
    // alternate between Lb and Lc
    int lcur = A_LA, loth = A_LB;
    for (int64_t i = x.len - 1; i >= 0; i--) {
      // u_{n0+i}: i forward steps from the checkpoint (up to `fuse` per
      // launch), the range shrinking to the interior at the last one
      int64_t u = buf(x.q, A_U0);
      int nw = 0;
      for (int64_t tt = 0; tt < i;) {
        const int lv = (int)std::min<int64_t>(fuse, i - tt);
        const int64_t dst = buf(x.q, (nw++ & 1) ? A_WB : A_WA);
        tt += lv;
        step(u, dst, i - tt, false, lv);
        u = dst;
      }
      Op o = B.blank(OP_AXPY, S_COMPUTE);   // g_c0 += lambda_{n0+i+1} * u_{n0+i}
      o.dev_dst = buf(x.q, A_G) + p.halo * (int64_t)pb;
      o.dev_src = buf(x.q, lcur) + p.halo * (int64_t)pb;
      o.dev_src2 = u + p.halo * (int64_t)pb;
      o.bytes = x.nz_int * (int64_t)pb;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
      step(buf(x.q, lcur), buf(x.q, loth), i, true, 1);   // lambda_{n0+i} = A^T lambda_{n0+i+1}
      lcur = loth;
      loth = lcur == A_LB ? A_LC : A_LB;
    }
    B.rec(S_COMPUTE, B.ev.out(x.q));
    return lcur;
  };
  auto issue_out = [&](int64_t g, int lres) {
    const Geo x = geo(g);
    std::vector<int> w{B.ev.out(x.q)};
    if (x.t > 0) {
      B.readers_of(x.sl->z0, x.sl->z1, &nb);
      for (int jj : nb) w.push_back(B.ev.h2d((x.t - 1) & 1, jj));
    }
    B.wait_all(S_OUT, w);
    for (int f = 0; f < 2; f++) {
      Op o = B.blank(OP_D2H, S_OUT);
      o.host_id = (int8_t)(f == 0 ? x.ldst : HOST_GRAD);
      o.dev_src = buf(x.q, f == 0 ? lres : A_G) + p.halo * (int64_t)pb;
      o.host_off = (int64_t)((size_t)x.sl->z0 * pb);
      o.bytes = x.nz_int * (int64_t)pb;
      o.slab = x.j;
      o.sweep = x.t;
      B.push(o);
    }
    B.rec(S_OUT, B.ev.free(x.q));
    B.rec(S_OUT, B.ev.d2h(x.t & 1, x.j));
  };
  int64_t next_in = 0, outs_issued = 0, computes_issued = 0;
  auto in_ready = [&](int64_t gi) {
    // a wait can only name an event already recorded: the shared-planes copy
    // of slab gi - NQ + 1 must have been issued
    if (gi >= NQ && has_share_copy(gi - NQ + 1) && computes_issued < gi - NQ + 2) return false;
    const int t = (int)(gi / ns);
    if (t == 0) return true;
    const Slab &sl = p.slabs[(size_t)(gi % ns)];
    B.writers_of(sl.l0, sl.l1, &nb);
    int jmax = 0;
    for (int jj : nb) jmax = std::max(jmax, jj);
    return (int64_t)(t - 1) * ns + jmax < outs_issued;
  };
  for (int64_t g = 0; g < total; g++) {
    while (next_in < total && next_in <= g + 1 && in_ready(next_in)) issue_in(next_in++);
    const int lres = issue_compute(g);
    computes_issued = g + 1;
    while (next_in < total && next_in <= g + 1 && in_ready(next_in)) issue_in(next_in++);
    issue_out(g, lres);
    outs_issued = g + 1;
  }
  B.push(B.blank(OP_SYNC, -1));
}

std::string dump_ops(const std::vector<Op> &ops) {
  static const char *names[] = {"H2D", "D2H", "DEC", "ENC", "STAR7", "WAVE", "AXPY", "REC", "WAIT", "SYNC",
                                "ZERO", "FUSED"};
  std::string out;
  char line[256];
  for (size_t i = 0; i < ops.size(); i++) {
    const Op &o = ops[i];
    if (o.type == OP_REC || o.type == OP_WAIT)
      snprintf(line, sizeof line, "%zu s%d %s ev=%d\n", i, o.stream, names[o.type], o.ev);
    else
      snprintf(line, sizeof line,
               "%zu s%d %s sweep=%d slab=%d src=%lld src2=%lld dst=%lld host=%d off=%lld bytes=%lld z=[%lld,%lld) lv=%d rate=%d\n",
               i, o.stream, names[o.type], o.sweep, o.slab, (long long)o.dev_src, (long long)o.dev_src2,
               (long long)o.dev_dst,
               o.host_id, (long long)o.host_off, (long long)o.bytes, (long long)o.z_lo, (long long)o.z_hi,
               (int)o.levels, (int)o.rate);
    out += line;
  }
  return out;
}

// ---------------------------------------------------------------------------
// happens-before checker
// ---------------------------------------------------------------------------
namespace {

struct Access {
  int res;          // 0 = device arena, 1 + host id = host store
  int64_t lo, hi;   // byte range
  bool write;
};

void accesses(const Plan &p, const Op &o, std::vector<Access> *a) {
  a->clear();
  auto dev = [&](int64_t off, int64_t bytes, bool w) {
    if (off >= 0 && bytes > 0) a->push_back({0, off, off + bytes, w});
  };
  switch (o.type) {
    case OP_H2D:
      a->push_back({1 + o.host_id, o.host_off, o.host_off + o.bytes, false});
      dev(o.dev_dst, o.bytes, true);
      break;
    case OP_D2H:
      dev(o.dev_src, o.bytes, false);
      a->push_back({1 + o.host_id, o.host_off, o.host_off + o.bytes, true});
      break;
    case OP_DEC:
      if (o.z_hi < 0) {
        dev(o.dev_src, o.bytes, false);
        dev(o.dev_dst, o.bytes, true);
      } else {
        // codes [0, bytes) from dev_src2 when set (shared layers left in the
        // previous slab's slot), the rest from dev_src at the same positions
        const size_t lb = o.rate > 0 ? coded_layer_bytes(p.in.nx, p.in.ny, o.rate) : p.layer_bytes;
        const int64_t lo = o.dev_src2 >= 0 ? o.bytes : 0;
        if (lo > 0) dev(o.dev_src2, lo, false);
        dev(o.dev_src + lo, (int64_t)((size_t)o.z_hi * lb) - lo, false);
        dev(o.dev_dst, (int64_t)((size_t)o.z_hi * 4 * p.plane_bytes), true);
      }
      break;
    case OP_ENC: {
      const size_t lb = o.rate > 0 ? coded_layer_bytes(p.in.nx, p.in.ny, o.rate) : p.layer_bytes;
      dev(o.dev_src, (int64_t)((size_t)o.z_hi * 4 * p.plane_bytes), false);
      dev(o.dev_dst, (int64_t)((size_t)o.z_hi * lb), true);
      break;
    }
    case OP_ZERO:
      dev(o.dev_dst, o.bytes, true);
      break;
    case OP_FUSED:
      // reads the slot's coded layers, writes the interior's codes
      dev(o.dev_src + o.z_lo * (int64_t)p.layer_bytes, (o.z_hi - o.z_lo) * (int64_t)p.layer_bytes, false);
      dev(o.dev_dst, o.bytes, true);
      break;
    case OP_AXPY:
      dev(o.dev_src, o.bytes, false);
      dev(o.dev_src2, o.bytes, false);
      dev(o.dev_dst, o.bytes, false);
      dev(o.dev_dst, o.bytes, true);
      break;
    case OP_STAR7:
    case OP_WAVE: {
      // reads planes [z_lo - r, z_hi + r) of the source (and the aux buffer),
      // writes [z_lo, z_hi) of the destination; WAVE also reads the destination
      int64_t pb = (int64_t)p.plane_bytes;
      const int64_t reach = (int64_t)p.r * o.levels;
      int64_t rlo = std::max<int64_t>(0, o.z_lo - reach), rhi = std::min<int64_t>(o.planes, o.z_hi + reach);
      dev(o.dev_src + rlo * pb, (rhi - rlo) * pb, false);
      if (o.dev_src2 >= 0) {
        const int64_t clo = std::max<int64_t>(0, o.z_lo - reach + p.r);
        const int64_t chi = std::min<int64_t>(o.planes, o.z_hi + reach - p.r);
        dev(o.dev_src2 + clo * pb, (chi - clo) * pb, false);
      }
      if (o.type == OP_WAVE) dev(o.dev_dst + o.z_lo * pb, (o.z_hi - o.z_lo) * pb, false);
      dev(o.dev_dst + o.z_lo * pb, (o.z_hi - o.z_lo) * pb, true);
      break;
    }
    default:
      break;
  }
}

}  // namespace

int64_t check_ops(const Plan &p, const std::vector<Op> &ops, std::string *why,
                  bool check_writeback) {
  const int NS = 3;
  // vector clock per stream, and the clock captured by each event's last record
  std::vector<std::vector<int64_t>> vc(NS, std::vector<int64_t>(NS, 0));
  std::vector<std::vector<int64_t>> evc(EventIds{(int)p.slabs.size()}.count() + 64,
                                        std::vector<int64_t>(NS, -1));
  std::vector<int> ev_recorded(evc.size(), 0);
  struct Stamp { int stream; int64_t clock; std::vector<int64_t> vc; size_t op; };
  std::vector<std::pair<Stamp, Access>> hist;
  std::vector<Access> acc;
  int64_t bad = 0;
  for (size_t i = 0; i < ops.size(); i++) {
    const Op &o = ops[i];
    if (o.type == OP_SYNC) {
      std::vector<int64_t> m(NS, 0);
      for (int s = 0; s < NS; s++)
        for (int q = 0; q < NS; q++) m[q] = std::max(m[q], vc[s][q]);
      for (int s = 0; s < NS; s++) vc[s] = m;
      continue;
    }
    const int s = o.stream;
    if (o.type == OP_REC) {
      evc[o.ev] = vc[s];
      ev_recorded[o.ev] = 1;
      continue;
    }
    if (o.type == OP_WAIT) {
      if (!ev_recorded[o.ev]) {
        bad++;
        if (why && why->empty()) *why = "wait on an event never recorded, op " + std::to_string(i);
        continue;
      }
      for (int q = 0; q < NS; q++) vc[s][q] = std::max(vc[s][q], evc[o.ev][q]);
      continue;
    }
    vc[s][s]++;
    Stamp st{s, vc[s][s], vc[s], i};
    accesses(p, o, &acc);
    for (const Access &a : acc) {
      for (const auto &h : hist) {
        const Access &b = h.second;
        if (b.res != a.res || b.hi <= a.lo || a.hi <= b.lo || (!a.write && !b.write)) continue;
        // ordered iff the earlier op's own clock is covered by this op's clock
        bool ordered = st.vc[h.first.stream] >= h.first.clock;
        if (!ordered) {
          bad++;
          if (why && why->empty()) {
            char buf[256];
            snprintf(buf, sizeof buf,
                     "ops %zu (stream %d, type %d) and %zu (stream %d, type %d) conflict on "
                     "resource %d [%lld,%lld)",
                     h.first.op, h.first.stream, (int)ops[h.first.op].type, i, s, (int)o.type,
                     a.res, (long long)std::max(a.lo, b.lo), (long long)std::min(a.hi, b.hi));
            *why = buf;
          }
        }
      }
    }
    for (const Access &a : acc) hist.push_back({st, a});
  }
  // every copy-in of sweep t must read the state sweep t-1 wrote (or the
  // loaded state when t = 0), never a plane this sweep has already written
  // back: with a single host level this is what makes the in-place update
  // correct.  Conflicting host accesses are ordered (checked above), and a
  // wait names only events recorded earlier in the list, so list order is
  // their execution order.
  if (check_writeback) {
    // per host level: sorted, disjoint [lo, hi) segments with the sweep that last wrote them
    struct Seg { int64_t lo, hi; int v; };
    std::vector<Seg> ver[2] = {{{0, (int64_t)p.host_level_bytes, -1}},
                               {{0, (int64_t)p.host_level_bytes, -1}}};
    for (size_t i = 0; i < ops.size(); i++) {
      const Op &o = ops[i];
      if ((o.type != OP_H2D && o.type != OP_D2H) || o.host_id < 0 || o.host_id > 1 || o.bytes <= 0)
        continue;
      std::vector<Seg> &vs = ver[o.host_id];
      const int64_t lo = o.host_off, hi = o.host_off + o.bytes;
      if (o.type == OP_H2D) {
        for (const Seg &g : vs)
          if (g.lo < hi && lo < g.hi && g.v != o.sweep - 1) {
            bad++;
            if (why && why->empty())
              *why = "op " + std::to_string(i) + " (sweep " + std::to_string(o.sweep) +
                     ") reads host bytes last written by sweep " + std::to_string(g.v);
            break;
          }
        continue;
      }
      std::vector<Seg> nv;
      for (const Seg &g : vs) {
        if (g.hi <= lo || hi <= g.lo) {
          nv.push_back(g);
          continue;
        }
        if (g.lo < lo) nv.push_back({g.lo, lo, g.v});
        if (hi < g.hi) nv.push_back({hi, g.hi, g.v});
      }
      nv.push_back({lo, hi, (int)o.sweep});
      std::sort(nv.begin(), nv.end(), [](const Seg &a, const Seg &b) { return a.lo < b.lo; });
      vs.swap(nv);
    }
  }
  // every sweep must write back each host store it writes, whole and once
  // (a level sized for a larger load rate is written up to the codes at the rate)
  const int64_t level_written =
      (p.coded && p.load_rate > p.in.rate)
          ? (int64_t)((size_t)(p.n_rw - 1) * p.host_field_bytes + (size_t)(p.in.nz / 4) * p.layer_bytes)
          : (int64_t)p.host_level_bytes;
  if (check_writeback) {
    int max_sweep = -1;
    for (const Op &o : ops) max_sweep = std::max(max_sweep, (int)o.sweep);
    for (int t = 0; t <= max_sweep; t++) {
      bool any = false;
      for (int id = 0; id < kHostStores; id++) {
        std::vector<std::pair<int64_t, int64_t>> rs;
        for (const Op &o : ops)
          if (o.type == OP_D2H && o.sweep == t && o.host_id == id)
            rs.push_back({o.host_off, o.host_off + o.bytes});
        if (rs.empty()) continue;
        if (id <= HOST_LEVEL1) any = true;
        std::sort(rs.begin(), rs.end());
        // a level is written whole; another store (a checkpoint) as one
        // contiguous range
        const int64_t from = id <= HOST_LEVEL1 ? 0 : rs.front().first;
        int64_t at = from;
        for (const auto &r : rs) {
          if (r.first != at) break;
          at = r.second;
        }
        if (id > HOST_LEVEL1 ? at != rs.back().second : at != level_written) {
          bad++;
          if (why && why->empty())
            *why = "sweep " + std::to_string(t) + " does not write back store " +
                   std::to_string(id) + " whole";
        }
      }
      if (!any) {
        bad++;
        if (why && why->empty()) *why = "sweep " + std::to_string(t) + " writes nothing back";
      }
    }
  }
  // everything must have been synchronised at the end
  if (ops.empty() || ops.back().type != OP_SYNC) {
    bad++;
    if (why && why->empty()) *why = "operation list does not end with a host sync";
  }
  return bad;
}

}  // namespace oc
