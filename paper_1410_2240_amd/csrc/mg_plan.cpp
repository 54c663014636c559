// Level plan and workspace layout (pure host C++; see mg_plan.h).
#include "mg_plan.h"

namespace mg {

namespace {

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  }
};

}  // namespace

int validate_dims(const int dims[3], int* n_out) {
  if (!dims) return -1;
  const int n = dims[0];
  if (dims[1] != n || dims[2] != n) return -1;
  if (n < 2 * kCoarsest || n > kMaxN) return -1;
  if ((n & (n - 1)) != 0) return -1;
  if (n_out) *n_out = n;
  return 0;
}

int build_plan(int n, int flags, Plan* plan) {
  const int d[3] = {n, n, n};
  if (validate_dims(d, nullptr) != 0 || !plan) return -1;
  if (flags < 0 || flags > (kFlagMixed | kFlagKrylov | kFlagDensity | kFlagFromRho)) return -1;
  const bool mixed = (flags & kFlagMixed) != 0;
  const bool density32 = mixed && n >= kDensity32MinN;   // the finest grid's FP32 density copy
  Plan p;
  p.n = n;
  p.flags = flags;
  Carver c;
  int L = 0;
  for (int m = n; m >= kCoarsest; m /= 2) ++L;
  p.levels = L;
  for (int l = 0; l < L; ++l) {
    LevelPlan& lv = p.lv[l];
    lv.n = n >> l;
    int q = 0;
    while ((1 << q) < lv.n) ++q;
    lv.log2n = q;
    const size_t cells = static_cast<size_t>(lv.n) * lv.n * lv.n;
    lv.bx = c.take(cells * 8);
    lv.by = c.take(cells * 8);
    lv.bz = c.take(cells * 8);
    lv.mask = c.take(cells);
    // level 0: f and p belong to the caller; t is the second buffer for p
    lv.f = l > 0 ? c.take(cells * 8) : kAbsent;
    lv.e = l > 0 ? c.take(cells * 8) : kAbsent;
    lv.t = c.take(cells * 8);
    // finest grid: the density form of the face coefficients (hierarchies built from rho)
    lv.rt = l == 0 ? c.take(cells * 8) : kAbsent;
    if (mixed) {
      if (l == 0 && density32 && (flags & kFlagFromRho)) {
        lv.bx32 = lv.by32 = lv.bz32 = kAbsent;
      } else {
        lv.bx32 = c.take(cells * 4);
        lv.by32 = c.take(cells * 4);
        lv.bz32 = c.take(cells * 4);
      }
      lv.f32 = c.take(cells * 4);   // level 0: the FP32 residual of each refinement step
      lv.e32 = c.take(cells * 4);
      lv.t32 = c.take(cells * 4);
      lv.rt32 = l == 0 && density32 ? c.take(cells * 4) : kAbsent;
    } else {
      lv.bx32 = lv.by32 = lv.bz32 = lv.f32 = lv.e32 = lv.t32 = kAbsent;
    }
  }
  if (flags & kFlagKrylov) {
    const size_t fine = static_cast<size_t>(n) * n * n * 8;
    p.kr = c.take(fine);
    p.kz = c.take(fine);
    p.kd = c.take(fine);
    p.kd2 = c.take(fine);
    p.kw = c.take(fine);
    if (plan_has_kr2(n, flags)) p.kr2 = c.take(fine);
    if (plan_has_kd3(n, flags)) p.kd3 = c.take(fine);
  }
  const size_t nc = static_cast<size_t>(kCoarsest) * kCoarsest * kCoarsest;
  p.pinv = c.take(nc * nc * 8);
  p.partials = c.take(static_cast<size_t>(kPartialSets) * kNumPartials * 8);
  p.scalars = c.take(32 * 8);
  p.counters = c.take(16 * 8);
  p.total = c.off;
  *plan = p;
  return 0;
}

int build_lane_plan(int n, int flags, Plan* plan) {
  Plan full;
  if (build_plan(n, flags, &full) != 0 || !plan) return -1;
  const bool mixed = (flags & kFlagMixed) != 0;
  Plan p;
  p.n = n;
  p.flags = flags;
  p.levels = full.levels;
  Carver c;
  for (int l = 0; l < p.levels; ++l) {
    LevelPlan& lv = p.lv[l];
    lv.n = full.lv[l].n;
    lv.log2n = full.lv[l].log2n;
    const size_t cells = static_cast<size_t>(lv.n) * lv.n * lv.n;
    lv.bx = lv.by = lv.bz = lv.mask = kAbsent;
    lv.bx32 = lv.by32 = lv.bz32 = kAbsent;
    lv.f = l > 0 ? c.take(cells * 8) : kAbsent;
    lv.e = l > 0 ? c.take(cells * 8) : kAbsent;
    lv.t = c.take(cells * 8);
    if (mixed) {
      lv.f32 = c.take(cells * 4);
      lv.e32 = c.take(cells * 4);
      lv.t32 = c.take(cells * 4);
    } else {
      lv.f32 = lv.e32 = lv.t32 = kAbsent;
    }
  }
  if (flags & kFlagKrylov) {
    const size_t fine = static_cast<size_t>(n) * n * n * 8;
    p.kr = c.take(fine);
    p.kz = c.take(fine);
    p.kd = c.take(fine);
    p.kd2 = c.take(fine);
    p.kw = c.take(fine);
    if (plan_has_kr2(n, flags)) p.kr2 = c.take(fine);
    if (plan_has_kd3(n, flags)) p.kd3 = c.take(fine);
  }
  p.pinv = kAbsent;
  p.partials = c.take(static_cast<size_t>(kPartialSets) * kNumPartials * 8);
  p.scalars = c.take(32 * 8);
  p.counters = kAbsent;
  p.total = c.off;
  *plan = p;
  return 0;
}

}  // namespace mg
