// Level plan and workspace layout of the multigrid solver (pure host C++).
//
// Every grid of the hierarchy halves the cell count per side of the one above it,
// from the finest N down to the 4^3 grid that is solved directly (section 3.1 keeps
// the face products on every grid, so each level stores its own three face arrays).
// This file only does arithmetic on sizes and offsets; it is compiled into the HIP
// library and, unchanged, into a host-only test program.
#pragma once

#include <cstddef>
#include <cstdint>

namespace mg {

constexpr int kCoarsest = 4;          // cells per side of the directly solved grid
constexpr int kMaxN = 1024;           // N^3 < 2^31: 32-bit cell indices throughout
constexpr int kMaxLevels = 10;        // 1024 -> 4
constexpr int kNumPartials = 16384;   // blocks of the two-pass reductions
constexpr size_t kAlign = 256;
constexpr int kPartialSets = 4;       // reductions that may be in flight together
constexpr int kFlagMixed = 1, kFlagKrylov = 2, kFlagDensity = 4, kFlagFromRho = 8;
// A mixed hierarchy's finest grid of this size and up keeps an FP32 copy of the density
// (the grids its one-pass and two-pass sweeps run on), from which the FP32 cycles form
// their finest faces; with kFlagFromRho it has no FP32 face arrays.
constexpr int kDensity32MinN = 64;

constexpr size_t kAbsent = static_cast<size_t>(-1);

struct LevelPlan {
  int n = 0;         // cells per side
  int log2n = 0;
  // FP64 arrays (byte offsets into the workspace; SIZE_MAX = absent)
  size_t bx = 0, by = 0, bz = 0;   // face coefficients
  size_t mask = 0;                 // uint8 activity
  size_t f = 0, e = 0;             // right-hand side / correction (levels >= 1)
  size_t t = 0;                    // second buffer for out-of-place sweeps
  size_t rt = kAbsent;             // level 0 only: rho on active cells, +inf elsewhere
  size_t rt32 = kAbsent;           // level 0, mixed only: the same in FP32
  // FP32 arrays (mixed precision only)
  size_t bx32 = 0, by32 = 0, bz32 = 0;
  size_t f32 = 0, e32 = 0, t32 = 0;
};

// the second residual kr2 and the third direction kd3 of a flexible-CG plan
inline bool plan_has_kr2(int n, int flags) {
  return (flags & kFlagKrylov) && !(flags & kFlagMixed) && (flags & kFlagFromRho) && n >= 256;
}
inline bool plan_has_kd3(int n, int flags) { return (flags & kFlagKrylov) && (flags & kFlagFromRho) && n >= 128; }

struct Plan {
  int n = 0;
  int levels = 0;
  int flags = 0;
  LevelPlan lv[kMaxLevels];
  // finest-grid FP64 vectors of the flexible-CG outer iteration (Krylov flag only):
  // residual, preconditioned residual, two directions (old and new), and A d; kr2, a
  // second residual, only for FP64 setups from rho on grids of 256^3 and up, whose
  // preconditioner's first pass forms the updated residual out of place; kd3, a third
  // direction, for setups from rho on grids of 128^3 and up, which update p every
  // second step (the direction of the step before is still needed then)
  size_t kr = kAbsent, kz = kAbsent, kd = kAbsent, kd2 = kAbsent, kw = kAbsent, kr2 = kAbsent, kd3 = kAbsent;
  size_t pinv = 0;       // (4^3)^2 doubles: pseudo-inverse of the coarsest operator
  size_t partials = 0;   // kPartialSets x kNumPartials doubles
  size_t scalars = 0;    // 32 doubles of device scalars
  size_t counters = 0;   // 16 int64 counters (setup validation and counts)
  size_t total = 0;      // bytes
};

// 0 if dims describe a supported cube (equal powers of two, 8..1024), else -1.
int validate_dims(const int dims[3], int* n_out);

// Fills `plan` for an N^3 grid and flags (bit 0 mixed precision, bit 1 flexible CG,
// bit 2 density coarsening, which needs no extra storage, bit 3 a setup from the
// density); returns 0, or -1 for unsupported N or flags.
int build_plan(int n, int flags, Plan* plan);

// The arrays one solve writes (every grid's right-hand side, correction and second
// buffers, the flexible-CG vectors, reduction partials and device scalars), laid out
// on their own: the scratch of one more right-hand side solved concurrently with the
// context's own.  Coefficients, masks and the pseudo-inverse are absent (kAbsent):
// they are read-only during a solve and shared.  Returns 0, or -1 as build_plan.
int build_lane_plan(int n, int flags, Plan* plan);

}  // namespace mg
