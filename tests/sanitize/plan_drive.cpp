// Drives the host planner (slab plan, arena carve-out, operation lists of the
// forward sweeps and of the adjoint's reverse sweeps, and the happens-before
// checker) over a sweep of configurations, for a build with AddressSanitizer
// and UndefinedBehaviorSanitizer: the 64-bit offset arithmetic of the carve-out
// and of the op builders must stay defined, and every op list must check
// race-free.  Exit status 0 = clean.
#include <cstdio>
#include <string>
#include <vector>

#include "oc_plan.h"

using namespace oc;

static int bad = 0;

static void forward(PlanInput in, int64_t sweeps) {
  Plan p;
  const int st = make_plan(in, &p);
  if (st != ST_OK) return;   // refused combinations are part of the sweep
  for (int steps_last = 1; steps_last <= in.k; steps_last++) {
    std::vector<Op> ops;
    build_ops(p, sweeps, steps_last, 0, 0, &ops);
    std::string why;
    if (check_ops(p, ops, &why) != 0) {
      std::fprintf(stderr, "race: nz=%lld k=%d S=%d R=%d fused=%d share=%d: %s\n", (long long)in.nz, in.k,
                   in.slab_planes, in.rate, (int)in.fused_codec, (int)in.share, why.c_str());
      bad++;
    }
    (void)dump_ops(ops);
  }
  if (ckpt_out_supported(p, 0) || ckpt_out_supported(p, 16)) {
    for (int rate : {0, 16}) {
      if (!ckpt_out_supported(p, rate)) continue;
      CkptOut ck;
      ck.rate = rate;
      std::vector<Op> ops;
      build_ops(p, sweeps, in.k, 0, 0, &ops, &ck);
      std::string why;
      if (check_ops(p, ops, &why) != 0) {
        std::fprintf(stderr, "race (checkpoint): %s\n", why.c_str());
        bad++;
      }
    }
  }
}

int main() {
  const int64_t shapes[][3] = {{16, 8, 8}, {40, 12, 16}, {44, 24, 40}, {36, 8, 12}, {28, 64, 60},
                               {9, 5, 7}};
  // the bench job's plan (512 x 512 x 2048, 512 MiB) in its main variants
  for (int rate : {0, 8, 16})
    for (int flags : {0, 2, 6, 10, 14}) {
      PlanInput in;
      in.nz = 2048;
      in.ny = 512;
      in.nx = 512;
      in.k = 4;
      in.slab_planes = 64;
      in.rate = rate;
      in.share = (flags & 2) != 0;
      in.in_place = (flags & 4) != 0;
      in.fused_codec = (flags & 8) != 0;
      in.budget = (size_t)512 << 20;
      forward(in, 2);
    }
  for (const auto &sh : shapes)
    for (int kind : {KIND_STAR7, KIND_WAVE25})
      for (int k : {1, 2, 3, 4, 5})
        for (int S : {0, 4, 8, 12, 64})
          for (int rate : {0, 1, 8, 16, 32})
            for (int flags = 0; flags < 16; flags++) {
              PlanInput in;
              in.nz = sh[0];
              in.ny = sh[1];
              in.nx = sh[2];
              in.kind = kind;
              in.k = k;
              in.slab_planes = S;
              in.rate = rate;
              in.single_buffer = (flags & 1) == 0;
              in.share = (flags & 2) != 0;
              in.in_place = (flags & 4) != 0;
              in.fused_codec = (flags & 8) != 0;
              in.c0_field = kind == KIND_STAR7 && (flags & 3) == 3;
              forward(in, 3);
            }
  // ring sizes and prefetch depths
  for (int slots = 2; slots <= kMaxSlots; slots++)
    for (int pre = 0; pre < slots; pre++) {
      PlanInput in;
      in.nz = 44;
      in.ny = 24;
      in.nx = 40;
      in.k = 4;
      in.slab_planes = 8;
      in.rate = 8;
      in.slots = slots;
      in.prefetch = pre;
      in.share = true;
      forward(in, 3);
      in.fused_codec = true;
      forward(in, 3);
    }
  // adjoint reverse sweeps
  for (const auto &sh : shapes) {
    if (sh[0] > 64) continue;
    for (int m : {1, 2, 4, 8})
      for (int rate : {0, 16})
        for (int share : {0, 1}) {
          PlanInput in;
          in.nz = sh[0];
          in.ny = sh[1];
          in.nx = sh[2];
          in.k = 1;
          in.rate = rate;
          in.share = share != 0;
          in.slab_planes = 8;
          AdjPlan a;
          if (make_adj_plan(in, m, 3 * m + 1, &a) != ST_OK) continue;
          std::vector<Op> ops;
          build_adjoint_ops(a, 0, &ops);
          std::string why;
          if (check_ops(a.g, ops, &why, false) != 0) {
            std::fprintf(stderr, "race (adjoint): %s\n", why.c_str());
            bad++;
          }
        }
  }
  if (bad) return 1;
  std::puts("plan_drive: clean");
  return 0;
}
