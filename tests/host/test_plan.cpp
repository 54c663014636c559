// Host-only checks of the level plan and workspace layout (built with g++, no GPU).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mg_plan.h"

namespace mg {
void symmetric_pinv(int n, std::vector<double>& a, double rtol, std::vector<double>& pinv);
bool graph_pinv(int n, const std::vector<double>& a, const std::vector<int>& component, double rtol,
                std::vector<double>& pinv);
}

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);     \
      ++failures;                                                  \
    }                                                              \
  } while (0)

struct Span {
  size_t off, len;
};

static void check_layout(int n, int flags) {
  mg::Plan p;
  CHECK(mg::build_plan(n, flags, &p) == 0);
  int L = 0;
  for (int m = n; m >= 4; m /= 2) ++L;
  CHECK(p.levels == L);
  CHECK(p.lv[L - 1].n == 4);
  std::vector<Span> spans;
  for (int l = 0; l < p.levels; ++l) {
    const mg::LevelPlan& a = p.lv[l];
    CHECK(a.n == (n >> l));
    CHECK((1 << a.log2n) == a.n);
    const size_t c = static_cast<size_t>(a.n) * a.n * a.n;
    spans.push_back({a.bx, c * 8});
    spans.push_back({a.by, c * 8});
    spans.push_back({a.bz, c * 8});
    spans.push_back({a.mask, c});
    spans.push_back({a.t, c * 8});
    if (l == 0) spans.push_back({a.rt, c * 8});
    else CHECK(a.rt == mg::kAbsent);
    if (l > 0) {
      spans.push_back({a.f, c * 8});
      spans.push_back({a.e, c * 8});
    } else {
      CHECK(a.f == mg::kAbsent && a.e == mg::kAbsent);
    }
    if (flags & 1) {
      const bool dens32 = l == 0 && n >= mg::kDensity32MinN;   // the finest grid's FP32 density copy
      if (dens32 && (flags & mg::kFlagFromRho)) {   // a setup from rho: no FP32 finest faces
        CHECK(a.bx32 == mg::kAbsent && a.by32 == mg::kAbsent && a.bz32 == mg::kAbsent);
      } else {
        for (size_t o : {a.bx32, a.by32, a.bz32}) spans.push_back({o, c * 4});
      }
      for (size_t o : {a.f32, a.e32, a.t32}) spans.push_back({o, c * 4});
      if (dens32) spans.push_back({a.rt32, c * 4});
      else CHECK(a.rt32 == mg::kAbsent);
    } else {
      CHECK(a.bx32 == mg::kAbsent && a.f32 == mg::kAbsent);
    }
  }
  const size_t fine = static_cast<size_t>(n) * n * n * 8;
  if (flags & 2) {
    for (size_t o : {p.kr, p.kz, p.kd, p.kd2, p.kw}) spans.push_back({o, fine});
  } else {
    CHECK(p.kr == mg::kAbsent && p.kw == mg::kAbsent);
  }
  // the second residual: FP64 flexible CG from rho on grids of 256^3 and up only
  if ((flags & 2) && !(flags & 1) && (flags & mg::kFlagFromRho) && n >= 256) spans.push_back({p.kr2, fine});
  else CHECK(p.kr2 == mg::kAbsent);
  // the third direction: flexible CG from rho on grids of 128^3 and up
  if ((flags & 2) && (flags & mg::kFlagFromRho) && n >= 128) spans.push_back({p.kd3, fine});
  else CHECK(p.kd3 == mg::kAbsent);
  spans.push_back({p.pinv, 64 * 64 * 8});
  spans.push_back({p.partials, static_cast<size_t>(mg::kPartialSets) * mg::kNumPartials * 8});
  spans.push_back({p.scalars, 32 * 8});
  spans.push_back({p.counters, 16 * 8});
  for (size_t i = 0; i < spans.size(); ++i) {
    CHECK(spans[i].off % mg::kAlign == 0);
    CHECK(spans[i].off + spans[i].len <= p.total);
    for (size_t j = i + 1; j < spans.size(); ++j) {
      const bool disjoint = spans[i].off + spans[i].len <= spans[j].off || spans[j].off + spans[j].len <= spans[i].off;
      CHECK(disjoint);
    }
  }
}

// The scratch of one concurrent right-hand side: exactly the arrays a solve writes, with
// the sizes the full plan gives them, disjoint and aligned; shared arrays absent.
static void check_lane_layout(int n, int flags) {
  mg::Plan full, p;
  CHECK(mg::build_plan(n, flags, &full) == 0);
  CHECK(mg::build_lane_plan(n, flags, &p) == 0);
  CHECK(p.levels == full.levels);
  CHECK(p.total % mg::kAlign == 0 && p.total < full.total);
  std::vector<Span> spans;
  for (int l = 0; l < p.levels; ++l) {
    const mg::LevelPlan& a = p.lv[l];
    CHECK(a.n == full.lv[l].n && a.log2n == full.lv[l].log2n);
    const size_t c = static_cast<size_t>(a.n) * a.n * a.n;
    for (size_t o : {a.bx, a.by, a.bz, a.mask, a.rt, a.rt32, a.bx32, a.by32, a.bz32}) CHECK(o == mg::kAbsent);
    spans.push_back({a.t, c * 8});
    if (l > 0) {
      spans.push_back({a.f, c * 8});
      spans.push_back({a.e, c * 8});
    } else {
      CHECK(a.f == mg::kAbsent && a.e == mg::kAbsent);
    }
    if (flags & 1) {
      for (size_t o : {a.f32, a.e32, a.t32}) spans.push_back({o, c * 4});
    } else {
      CHECK(a.f32 == mg::kAbsent && a.e32 == mg::kAbsent && a.t32 == mg::kAbsent);
    }
  }
  const size_t fine = static_cast<size_t>(n) * n * n * 8;
  if (flags & 2) {
    for (size_t o : {p.kr, p.kz, p.kd, p.kd2, p.kw}) spans.push_back({o, fine});
  } else {
    CHECK(p.kr == mg::kAbsent && p.kw == mg::kAbsent);
  }
  // the second residual: FP64 flexible CG from rho on grids of 256^3 and up only
  if ((flags & 2) && !(flags & 1) && (flags & mg::kFlagFromRho) && n >= 256) spans.push_back({p.kr2, fine});
  else CHECK(p.kr2 == mg::kAbsent);
  // the third direction: flexible CG from rho on grids of 128^3 and up
  if ((flags & 2) && (flags & mg::kFlagFromRho) && n >= 128) spans.push_back({p.kd3, fine});
  else CHECK(p.kd3 == mg::kAbsent);
  CHECK(p.pinv == mg::kAbsent && p.counters == mg::kAbsent);
  spans.push_back({p.partials, static_cast<size_t>(mg::kPartialSets) * mg::kNumPartials * 8});
  spans.push_back({p.scalars, 32 * 8});
  for (size_t i = 0; i < spans.size(); ++i) {
    CHECK(spans[i].off != mg::kAbsent);
    CHECK(spans[i].off % mg::kAlign == 0);
    CHECK(spans[i].off + spans[i].len <= p.total);
    for (size_t j = i + 1; j < spans.size(); ++j) {
      const bool disjoint = spans[i].off + spans[i].len <= spans[j].off || spans[j].off + spans[j].len <= spans[i].off;
      CHECK(disjoint);
    }
  }
}

int main() {
  const int good[3] = {64, 64, 64};
  int n = 0;
  CHECK(mg::validate_dims(good, &n) == 0 && n == 64);
  const int bad[][3] = {{64, 64, 32}, {48, 48, 48}, {4, 4, 4}, {2048, 2048, 2048}, {0, 0, 0}, {-8, -8, -8}};
  for (const auto& d : bad) CHECK(mg::validate_dims(d, nullptr) != 0);
  CHECK(mg::validate_dims(nullptr, nullptr) != 0);
  mg::Plan p;
  CHECK(mg::build_plan(64, 16, &p) != 0);
  CHECK(mg::build_plan(64, -1, &p) != 0);
  for (int m : {8, 16, 64, 256})
    for (int fl : {0, 1, 2, 3, 8, 9, 10, 11}) {
      check_layout(m, fl);
      check_lane_layout(m, fl);
    }
  CHECK(mg::build_lane_plan(48, 0, &p) != 0);
  CHECK(mg::build_lane_plan(64, 16, &p) != 0);
  // a mixed setup from rho on a grid of 64^3 and up leaves out the FP32 finest faces
  {
    mg::Plan pa, pb;
    for (int m : {64, 1024}) {
      CHECK(mg::build_plan(m, 1, &pa) == 0 && mg::build_plan(m, 1 | 8, &pb) == 0);
      const size_t faces = 3 * static_cast<size_t>(m) * m * m * 4;
      CHECK(pa.total - pb.total >= faces && pa.total - pb.total < faces + 3 * mg::kAlign);
    }
    CHECK(mg::build_plan(32, 1, &pa) == 0 && mg::build_plan(32, 1 | 8, &pb) == 0 && pa.total == pb.total);
    CHECK(mg::build_plan(256, 8, &pa) == 0 && mg::build_plan(256, 0, &pb) == 0 && pa.total == pb.total);
  }
  // density coarsening needs no storage of its own
  {
    mg::Plan pa, pb;
    CHECK(mg::build_plan(64, 3, &pa) == 0 && mg::build_plan(64, 7, &pb) == 0 && pa.total == pb.total);
  }
  // 1024^3 FP64: three FP64 face arrays, the mask and the second buffer on the finest grid
  CHECK(mg::build_plan(1024, 0, &p) == 0);
  const double fine = 1024.0 * 1024 * 1024 * (3 * 8 + 1 + 8 + 8);
  // coarse grids add 1/7 of that plus their right-hand side and correction
  CHECK(p.total > fine && p.total < 1024.0 * 1024 * 1024 * 49);
  // pseudo-inverse of a symmetric singular matrix: A A+ A = A
  std::vector<double> a = {2, -1, -1, -1, 2, -1, -1, -1, 2}, pinv;
  std::vector<double> a0 = a;
  mg::symmetric_pinv(3, a, 1e-12, pinv);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) s += a0[r * 3 + k] * pinv[k * 3 + l] * a0[l * 3 + c];
      CHECK(std::abs(s - a0[r * 3 + c]) < 1e-12);
    }
  // pinv of diag(2, 4) with a zero eigenvalue block
  std::vector<double> d = {2, 0, 0, 0, 4, 0, 0, 0, 0};
  mg::symmetric_pinv(3, d, 1e-12, pinv);
  CHECK(std::abs(pinv[0] - 0.5) < 1e-15 && std::abs(pinv[4] - 0.25) < 1e-15 && pinv[8] == 0.0);
  // graph pseudo-inverse: two components {0,1,2} and {3,4} plus an inactive cell 5
  {
    const int n = 6;
    std::vector<double> g(n * n, 0.0);
    auto edge = [&](int a, int b, double w) {
      g[a * n + b] += w; g[b * n + a] += w; g[a * n + a] -= w; g[b * n + b] -= w;
    };
    edge(0, 1, 2.0); edge(1, 2, 1000.0); edge(0, 2, 0.5); edge(3, 4, 3.0);
    std::vector<int> comp = {0, 0, 0, 1, 1, -1};
    std::vector<double> pg, pj, gj = g;
    CHECK(mg::graph_pinv(n, g, comp, 1e-14, pg));
    mg::symmetric_pinv(n, gj, 1e-12, pj);
    for (int i = 0; i < n * n; ++i) CHECK(std::abs(pg[i] - pj[i]) < 1e-12);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
  return failures ? 1 : 0;
}
